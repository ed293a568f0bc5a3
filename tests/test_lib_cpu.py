"""Host-side checks of the C ABI (no GPU needed): exports, configuration
space, argument validation on a host-only handle."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(kt_[a-z0-9_]+)\s*\(", txt))
    return names


def test_every_declared_symbol_is_exported(kt):
    L = ctypes.CDLL(kt.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header(kt):
    assert _declared() <= set(kt._SIGS) | {"kt_abi_version"}


def test_config_space(kt):
    from paper_2008_13145_amd import codegen
    h = kt.Handle(-1)
    cfgs = h.configs()
    assert len(cfgs) == 164
    assert cfgs == codegen.f32_configs()
    by_t = {t: sum(1 for c in cfgs if c[2] == t) for t in (1, 2, 4, 8)}
    assert by_t == {1: 60, 2: 52, 4: 36, 8: 16}
    for (bm, bn, t, bk) in cfgs:
        assert bm % (8 * t) == 0 and bn % (8 * t) == 0 and 1 <= bm * bn // (64 * t * t) <= 16
        assert bk in (8, 16, 32, 64)
    # every configuration is compiled for every layout in the full build
    assert all(h.config_compiled(i, ta, tb) for i in range(164) for ta, tb in synth.LAYOUTS)
    # the configuration of the single-GEMM workload (64x64 tile, 4x4 thread tile, BK 16)
    assert (64, 64, 4, 16) in cfgs


def test_low_precision_config_spaces(kt):
    """BF16 and FP8 spaces: the library's tables equal the generator's; the
    MFMA depth divides every K tile (16 / 32 for BF16 32x32 / 16x16 blocks,
    64 / 128 for FP8); every double-buffered stage fits the 160 KiB LDS; ids
    0..67 are the 32x32-block configurations and the 16x16-block (t = 2)
    ones follow; all are compiled for every layout."""
    from paper_2008_13145_amd import codegen
    h = kt.Handle(-1)
    for dt, eb, gen, n, depth32, depth16 in ((kt.BF16, 2, codegen.bf16_configs, 98, 16, 32),
                                             (kt.FP8E4M3, 1, codegen.fp8_configs, 83, 64, 128)):
        cfgs = h.configs(dt)
        assert cfgs == gen() and len(cfgs) == n
        assert all(c[2] >= 4 for c in cfgs[:68]) and all(c[2] == 2 for c in cfgs[68:])
        for (bm, bn, t, bk) in cfgs:
            wt = 8 * t
            assert bm % wt == 0 and bn % wt == 0 and 1 <= (bm // wt) * (bn // wt) <= 16
            assert bk % (depth16 if t == 2 else depth32) == 0
            assert 2 * (bm + bn) * (bk * eb + 16) <= 160 * 1024
        assert len(set(cfgs)) == n
        assert all(h.config_compiled(i, ta, tb, dtype=dt) for i in range(n) for ta, tb in synth.LAYOUTS)


def test_host_handle_rejects_gpu_work(kt):
    h = kt.Handle(-1)
    s = kt.shape(8, 8, 8)
    st = h.L.kt_gemm(h.h, 0, ctypes.byref(s), 1.0, None, 8, 0, None, 8, 0, 0.0, None, 8, 0,
                     None, None, 0, None)
    assert st == -1 and "device" in h.L.kt_last_error(h.h).decode()
    with pytest.raises(kt.KtError):
        h.get_config(164)
    with pytest.raises(kt.KtError):
        h.get_kernel(-1)
    with pytest.raises(kt.KtError):
        h.get_config(-1)


def test_create_rejects_bad_device(kt):
    with pytest.raises(kt.KtError):
        kt.Handle(-7)


def test_abi_version(kt):
    assert kt.lib().kt_abi_version() == 111


def test_kernel_ids(kt):
    """Kernels = configurations, then the split-K variants the generator
    defines (per tile of SPLIT_TILES -- square edges 16..128, then 16 x 128
    and 128 x 16: deepest K tile, then most waves; slices 2, 4, 8, 16);
    out-of-range ids are refused; the workspace a variant needs follows its
    slices and the 256 MiB cap."""
    from paper_2008_13145_amd import codegen
    h = kt.Handle(-1)
    for dt, gen in ((kt.F32, codegen.f32_configs), (kt.BF16, codegen.bf16_configs),
                    (kt.FP8E4M3, codegen.fp8_configs)):
        cfgs = gen()
        ks = h.kernels(dt)
        tiles = list(codegen.SPLIT_TILES)
        assert ks == codegen.kernels(cfgs) and len(ks) == len(cfgs) + 4 * len(tiles)
        for v in range(len(cfgs), len(ks)):
            k, base = h.get_kernel(v, dt)
            assert k[:4] == cfgs[base] and k[4] == (2, 4, 8, 16)[(v - len(cfgs)) % 4]
            assert (k[0], k[1]) == tiles[(v - len(cfgs)) // 4]
            same_tile = [c for c in cfgs if (c[0], c[1]) == (k[0], k[1])]
            assert k[3] == max(c[3] for c in same_tile)
            assert k[2] == min(c[2] for c in same_tile if c[3] == k[3])
            assert all(h.config_compiled(v, ta, tb, dtype=dt) for ta, tb in synth.LAYOUTS)
        with pytest.raises(kt.KtError):
            h.get_kernel(len(ks), dt)
    assert {k[:4] for k in h.kernels()[164:]} == {(16, 16, 1, 64), (32, 32, 1, 64),
                                                  (64, 64, 2, 64), (128, 128, 4, 64),
                                                  (16, 128, 2, 64), (128, 16, 2, 64)}
    v8 = next(v for v, k in enumerate(h.kernels()) if k[4] == 8)
    assert h.kernel_workspace_bytes(100, 50, 1000, 2, id=v8) == 8 * 2 * 100 * 50 * 4
    assert h.kernel_workspace_bytes(100, 50, 129, 2, id=v8) == -(-3 * 2 * 100 * 50 * 4 // 256) * 256
    assert h.kernel_workspace_bytes(4096, 4096, 8192, 1, id=v8) == 0
    with pytest.raises(kt.KtError):
        h.kernel_workspace_bytes(8, 8, 8, id=len(h.kernels()))


def test_sweep_workspace_query(kt):
    n = kt.Handle.sweep_workspace_bytes([(100, 200, 300, 2, 0, 1)])
    # A 2*100*300 + B 2*300*200 + C 2*100*200 floats, each region 256-aligned, plus scale slot
    assert n >= 4 * (60000 + 120000 + 40000)
    assert n % 256 == 0


def test_splitk_workspace_query_and_host_handle(kt):
    # splits * batch * M * N floats, 256-aligned; one slice needs none
    assert kt.Handle.splitk_workspace_bytes(100, 70, 5000, 3, 8) == -(-8 * 3 * 100 * 70 * 4 // 256) * 256
    assert kt.Handle.splitk_workspace_bytes(100, 70, 5000, 3, 1) == 0
    for bad in (65, -2):
        with pytest.raises(kt.KtError):
            kt.Handle.splitk_workspace_bytes(100, 70, 5000, 3, bad)
    # automatic (0): bounded by 64 planes and by 4096 tiles of the largest area
    assert kt.Handle.splitk_workspace_bytes(100, 70, 5000, 3, 0) == -(-64 * 3 * 100 * 70 * 4 // 256) * 256
    assert kt.Handle.splitk_workspace_bytes(4096, 4096, 5000, 1, 0) == 4096 * 256 * 256 * 4
    h = kt.Handle(-1)
    s = kt.shape(8, 8, 512)
    st = h.L.kt_gemm_splitk(h.h, 0, ctypes.byref(s), 4, 1.0, None, 512, 0, None, 8, 0, 0.0, None, 8,
                            0, None, None, 0, None, 0, None, None)
    assert st == -1 and "device" in h.L.kt_last_error(h.h).decode()


def test_conv_queries(kt):
    """The GEMM a convolution runs and its workspace (host-only queries)."""
    cs = kt.conv_shape(2, 224, 224, 3, 64)
    assert kt.Handle.conv_gemm_shape(cs, kt.CONV_IM2COL) == (2 * 224 * 224, 64, 27, 1, 0, 0)
    assert kt.Handle.conv_gemm_shape(cs, kt.CONV_WINOGRAD) == (2 * 112 * 112, 64, 3, 16, 0, 0)
    assert kt.Handle.conv_workspace_bytes(cs, kt.CONV_IM2COL) == 2 * 224 * 224 * 27 * 4
    T = 2 * 112 * 112
    a = lambda v: -(-v // 256) * 256
    assert kt.Handle.conv_workspace_bytes(cs, kt.CONV_WINOGRAD) == (a(16 * T * 3 * 4) + a(16 * 3 * 64 * 4)
                                                                   + a(16 * T * 64 * 4))
    # a 1x1 filter with stride 1 and no padding multiplies x itself: no patch matrix
    fc = kt.conv_shape(1, 1, 1, 25088, 4096, 1, 1, 1, 0)
    assert kt.Handle.conv_gemm_shape(fc, kt.CONV_IM2COL) == (1, 4096, 25088, 1, 0, 0)
    assert kt.Handle.conv_workspace_bytes(fc, kt.CONV_IM2COL) == 0
    assert kt.Handle.conv_workspace_bytes(fc, kt.CONV_IM2COL, 8) == -(-8 * 4096 * 4 // 256) * 256
    with pytest.raises(kt.KtError):
        kt.Handle.conv_workspace_bytes(kt.conv_shape(1, 8, 8, 4, 4), kt.CONV_WINOGRAD, 2)
    # strided / larger filters: im2col only
    cs = kt.conv_shape(1, 15, 15, 8, 8, 5, 5, 2, 2)
    assert kt.Handle.conv_gemm_shape(cs, kt.CONV_IM2COL) == (64, 8, 200, 1, 0, 0)
    with pytest.raises(kt.KtError):
        kt.Handle.conv_gemm_shape(cs, kt.CONV_WINOGRAD)
    with pytest.raises(kt.KtError):
        kt.Handle.conv_workspace_bytes(kt.conv_shape(1, 8, 8, 0, 4), kt.CONV_IM2COL)
    h = kt.Handle(-1)
    with pytest.raises(kt.KtError):
        h.conv2d(kt.CONV_IM2COL, kt.conv_shape(1, 8, 8, 4, 4), 8, 8, None, False, 8, 8, 1 << 20)


def test_pipeline_query(kt):
    """Which pipeline a call takes (host only): LDS DMA when every
    row starts on a 16-byte boundary and the contiguous extents are whole
    16-byte chunks, or with whole rows promised, at least one chunk reaching
    within the leading dimension."""
    BF16, FP8 = kt.BF16, kt.FP8E4M3
    h = kt.Handle(-1)
    shp = kt.shape(64, 64, 64)
    assert h.dma_pipeline(BF16, shp, 0x1000, 64, 0, 0x2000, 64, 0)
    assert h.dma_pipeline(0, shp, 0x1000, 64, 0, 0x2000, 64, 0)              # FP32 too
    assert not h.dma_pipeline(0, shp, 0x1000, 66, 0, 0x2000, 64, 0)          # FP32, odd rows
    assert not h.dma_pipeline(BF16, shp, 0x1008, 64, 0, 0x2000, 64, 0)       # base
    assert not h.dma_pipeline(BF16, shp, 0x1000, 68, 0, 0x2000, 64, 0)       # lda
    assert not h.dma_pipeline(BF16, kt.shape(64, 64, 60), 0x1000, 64, 0, 0x2000, 64, 0)
    assert not h.dma_pipeline(BF16, kt.shape(64, 60, 64), 0x1000, 64, 0, 0x2000, 64, 0)
    assert h.dma_pipeline(BF16, kt.shape(60, 64, 64, 1, 0, 1), 0x1000, 64, 0, 0x2000,
                                     64, 0)                                             # M free
    assert not h.dma_pipeline(FP8, shp, 0x1000, 72, 0, 0x2000, 64, 0)
    assert not h.dma_pipeline(BF16, kt.shape(64, 64, 64, 2), 0x1000, 64, 4100, 0x2000,
                                         64, 4096)                                      # stride
    ragged = kt.shape(64, 60, 61)                       # K and N off 16-byte chunks
    assert not h.dma_pipeline(BF16, ragged, 0x1000, 64, 0, 0x2000, 64, 0)
    h.set_full_rows(True)
    assert h.dma_pipeline(BF16, ragged, 0x1000, 64, 0, 0x2000, 64, 0)
    assert not h.dma_pipeline(BF16, ragged, 0x1000, 64, 0, 0x2000, 56, 0)   # ldb short of 64
    assert not h.dma_pipeline(BF16, kt.shape(64, 60, 5), 0x1000, 8, 0, 0x2000, 64, 0)
    h.set_full_rows(False)
    assert not h.dma_pipeline(BF16, ragged, 0x1000, 64, 0, 0x2000, 64, 0)
    h.close()
