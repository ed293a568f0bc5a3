"""GPU parity of the convolution layers (im2col and Winograd F(2x2,3x3)
around the FP32 GEMM, 2x2 max pooling) against the FP64 direct-convolution
oracle.

Tolerances (per element):
* im2col: the GEMM bound with K = R*S*Cin, 1e-5 * sqrt(K) * max|x| * max|w|,
  plus 2^-22 * (|y| + |bias|) for the bias addition.
* Winograd: the transformed operands grow by at most 4 (input: sums of four
  values) and 2.25 (filter: two averages of three), the products are summed
  over Cin by the GEMM (1e-5 * sqrt(Cin) per unit of magnitude) and the
  output transform adds nine of them: 9 * 9 * 1e-5 * sqrt(Cin) <= 1e-3 *
  sqrt(Cin), times max|x| * max|w|, plus the bias term.
* Small integers: every transformed value (multiples of 1/4), product and
  sum is exact in FP32, so both algorithms equal the oracle bit for bit.
* Max pooling selects values: bit for bit."""
import math

import numpy as np
import pytest

import synth
from oracle import conv as oc

pytestmark = pytest.mark.gpu

IM2COL, WINO = 0, 1


def _data(n, H, W, C, O, R, S, seed):
    x = synth.uniform_operand(synth.operand_seed(seed, 0), n * H * W * C).reshape(n, H, W, C)
    w = synth.uniform_operand(synth.operand_seed(seed, 1), R * S * C * O).reshape(R, S, C, O)
    b = synth.uniform_operand(synth.operand_seed(seed, 2), O)
    return x, w, b


def _run(h, torch, algo, cs, x, w, b, relu, cfg, splits=1):
    import paper_2008_13145_amd as kt
    Ho, Wo = oc.out_size(cs.H, cs.R, cs.stride, cs.pad), oc.out_size(cs.W, cs.S, cs.stride, cs.pad)
    ws_bytes = kt.Handle.conv_workspace_bytes(cs, algo, splits)
    ws = torch.empty(max(ws_bytes, 4), dtype=torch.uint8, device="cuda")
    dx = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    dw = torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda()
    db = None if b is None else torch.from_numpy(np.ascontiguousarray(b, np.float32)).cuda()
    dy = torch.full((cs.n, max(Ho, 0), max(Wo, 0), cs.Cout), float("nan"), device="cuda")
    h.conv2d(algo, cs, dx, dw, db, relu, dy, ws, ws_bytes, config_id=cfg, splits=splits)
    torch.cuda.synchronize()
    return dy.cpu().numpy()


def _tol(algo, x, w, b, ref, cs):
    xm, wm = float(np.abs(x).max()), float(np.abs(w).max())
    if algo == IM2COL:
        base = 1e-5 * math.sqrt(cs.R * cs.S * cs.Cin) * xm * wm
    else:
        base = 1e-3 * math.sqrt(cs.Cin) * xm * wm
    bt = 0.0 if b is None else np.abs(b)
    return base + 2.0 ** -22 * (np.abs(ref) + bt)


IM2COL_CASES = [
    (2, 13, 11, 3, 16, 3, 3, 1, 1),
    (1, 20, 17, 35, 70, 3, 3, 2, 1),
    (1, 9, 9, 8, 5, 5, 5, 1, 2),
    (3, 6, 7, 64, 33, 1, 1, 1, 0),
    (1, 28, 28, 64, 128, 3, 3, 1, 1),
]


@pytest.mark.parametrize("case", IM2COL_CASES)
def test_im2col_parity(gpu, case):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cs = kt.conv_shape(*case)
    x, w, b = _data(*case[:7], seed=300 + sum(case))
    for cfg, relu, bias in ((h.configs().index((64, 64, 4, 16)), True, b),
                            (h.configs().index((32, 32, 2, 32)), False, None)):
        ref = oc.conv2d(x, w, bias, cs.stride, cs.pad, relu)
        got = _run(h, torch, IM2COL, cs, x, w, bias, relu, cfg)
        assert got.shape == ref.shape
        assert np.all(np.abs(got - ref) <= _tol(IM2COL, x, w, bias, ref, cs)), (cfg, relu)


WINO_CASES = [
    (2, 13, 11, 3, 16, 1),
    (1, 14, 14, 64, 128, 1),
    (1, 7, 9, 32, 48, 0),
    (2, 5, 4, 17, 9, 1),
    (1, 56, 56, 128, 64, 1),
]


@pytest.mark.parametrize("case", WINO_CASES)
def test_winograd_parity(gpu, case):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    n, H, W, C, O, pad = case
    cs = kt.conv_shape(n, H, W, C, O, 3, 3, 1, pad)
    x, w, b = _data(n, H, W, C, O, 3, 3, seed=500 + sum(case))
    assert h.conv_gemm_shape(cs, WINO) == (n * -(-(H + 2 * pad - 2) // 2) * -(-(W + 2 * pad - 2) // 2),
                                           O, C, 16, 0, 0)
    for cfg, relu, bias in ((h.configs().index((64, 64, 4, 16)), True, b),
                            (h.configs().index((128, 128, 8, 8)), False, None)):
        ref = oc.conv2d(x, w, bias, 1, pad, relu)
        got = _run(h, torch, WINO, cs, x, w, bias, relu, cfg)
        assert got.shape == ref.shape
        assert np.all(np.abs(got - ref) <= _tol(WINO, x, w, bias, ref, cs)), (cfg, relu)


@pytest.mark.parametrize("algo", [IM2COL, WINO])
def test_small_integers_bitwise(gpu, algo):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    rng = np.random.default_rng(algo)
    n, H, W, C, O = 2, 15, 10, 24, 40
    x = rng.integers(-3, 4, size=(n, H, W, C)).astype(np.float32)
    w = rng.integers(-2, 3, size=(3, 3, C, O)).astype(np.float32)
    b = rng.integers(-4, 5, size=O).astype(np.float32)
    cs = kt.conv_shape(n, H, W, C, O)
    ref = oc.conv2d(x, w, b, 1, 1, True)
    got = _run(h, torch, algo, cs, x, w, b, True, h.configs().index((64, 64, 4, 16)))
    assert np.array_equal(got, ref.astype(np.float32))


def test_maxpool_bitwise(gpu):
    h, torch = gpu
    for (n, H, W, C) in ((2, 8, 6, 5), (1, 9, 7, 64), (3, 1, 4, 2), (1, 224, 224, 64)):
        x = synth.uniform_operand(77 + H, n * H * W * C).reshape(n, H, W, C)
        dx = torch.from_numpy(x).cuda()
        dy = torch.full((n, H // 2, W // 2, C), float("nan"), device="cuda")
        h.maxpool2x2(dx, n, H, W, C, dy)
        torch.cuda.synchronize()
        assert np.array_equal(dy.cpu().numpy(), oc.maxpool2x2(x))


def test_vgg_block_layer_by_layer(gpu):
    """The first VGG16 block at 32x32 (conv 3->64, conv 64->64, ReLU, pool)
    with both algorithms: each layer against the oracle applied to that
    layer's GPU input."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cfg = h.configs().index((64, 64, 4, 16))
    for algo in (IM2COL, WINO):
        act = synth.uniform_operand(41, 32 * 32 * 3).reshape(1, 32, 32, 3)
        C = 3
        for li, O in enumerate((64, 64)):
            _, w, b = _data(1, 1, 1, C, O, 3, 3, seed=60 + li)
            cs = kt.conv_shape(1, 32, 32, C, O)
            got = _run(h, torch, algo, cs, act, w, b, True, cfg)
            ref = oc.conv2d(act, w, b, 1, 1, True)
            assert np.all(np.abs(got - ref) <= _tol(algo, act, w, b, ref, cs)), (algo, li)
            act, C = got, O
        dx = torch.from_numpy(act).cuda()
        dy = torch.empty((1, 16, 16, 64), device="cuda")
        h.maxpool2x2(dx, 1, 32, 32, 64, dy)
        torch.cuda.synchronize()
        assert np.array_equal(dy.cpu().numpy(), oc.maxpool2x2(act))


def test_conv_edge_cases(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cfg = h.configs().index((32, 32, 2, 32))
    # empty batch and an empty output (H + 2 pad < R) are no-ops
    for cs in (kt.conv_shape(0, 8, 8, 4, 4), kt.conv_shape(1, 1, 1, 4, 4, 5, 5, 1, 1)):
        for algo in (IM2COL,) if cs.R == 5 else (IM2COL, WINO):
            ws = torch.empty(256, dtype=torch.uint8, device="cuda")
            y = torch.zeros(16, device="cuda")
            x = torch.zeros(16, device="cuda")
            h.conv2d(algo, cs, x, x, None, False, y, ws, 256, config_id=cfg)
    # Winograd needs 3x3 stride 1
    for cs in (kt.conv_shape(1, 8, 8, 4, 4, 5, 5, 1, 2), kt.conv_shape(1, 8, 8, 4, 4, 3, 3, 2, 1)):
        with pytest.raises(kt.KtError) as e:
            kt.Handle.conv_workspace_bytes(cs, WINO)
        assert e.value.status == -2
    # a short workspace is rejected before any launch
    cs = kt.conv_shape(1, 8, 8, 4, 4)
    x = torch.zeros((1, 8, 8, 4), device="cuda")
    w = torch.zeros((3, 3, 4, 4), device="cuda")
    y = torch.full((1, 8, 8, 4), 5.0, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    for algo in (IM2COL, WINO):
        with pytest.raises(kt.KtError) as e:
            h.conv2d(algo, cs, x, w, None, False, y, ws, 256, config_id=cfg)
        assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((y == 5.0).all())


@pytest.mark.parametrize("case,splits", [
    ((1, 1, 1, 2048, 300, 1, 1, 1, 0), 0),     # a fully connected layer: M = 1, automatic split
    ((1, 1, 1, 4096, 1000, 1, 1, 1, 0), 8),
    ((3, 6, 7, 64, 33, 1, 1, 1, 0), 1),        # pointwise, no patch matrix
    ((1, 10, 10, 64, 32, 3, 3, 1, 1), 3),      # 3x3 through split-K
])
def test_im2col_split_k_and_pointwise(gpu, case, splits):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cs = kt.conv_shape(*case)
    x, w, b = _data(*case[:7], seed=800 + sum(case))
    cfg = h.configs().index((64, 64, 4, 16))
    for relu, bias in ((True, b), (False, None)):
        ref = oc.conv2d(x, w, bias, cs.stride, cs.pad, relu)
        got = _run(h, torch, IM2COL, cs, x, w, bias, relu, cfg, splits)
        assert np.all(np.abs(got - ref) <= _tol(IM2COL, x, w, bias, ref, cs)), (relu, splits)
    with pytest.raises(kt.KtError) as e:
        kt.Handle.conv_workspace_bytes(kt.conv_shape(1, 8, 8, 4, 4), WINO, 2)
    assert e.value.status == -2


def test_graph_captured_stack_matches_eager(gpu):
    """A small stack (Winograd 3x3 conv + ReLU, 2x2 pool, fully connected
    layer through automatic split-K) captured in one graph: three replays,
    with eager work on other data between them, each equal bit for bit to
    the eager result and within the oracle bound."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    cfg = h.configs().index((64, 64, 4, 16))
    c1 = kt.conv_shape(1, 16, 16, 8, 32)
    fc = kt.conv_shape(1, 1, 1, 8 * 8 * 32, 100, 1, 1, 1, 0)
    x, w1, b1 = _data(1, 16, 16, 8, 32, 3, 3, seed=91)
    _, w2, b2 = _data(1, 1, 1, 8 * 8 * 32, 100, 1, 1, seed=92)
    ws_bytes = max(kt.Handle.conv_workspace_bytes(c1, WINO), kt.Handle.conv_workspace_bytes(fc, IM2COL, 0))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    dx = torch.from_numpy(x).cuda()
    dw1, db1 = torch.from_numpy(w1).cuda(), torch.from_numpy(b1).cuda()
    dw2, db2 = torch.from_numpy(w2).cuda(), torch.from_numpy(b2).cuda()
    a1 = torch.empty((1, 16, 16, 32), device="cuda")
    p1 = torch.empty((1, 8, 8, 32), device="cuda")
    y = torch.empty((1, 1, 1, 100), device="cuda")

    def net(inp, st):
        h.conv2d(WINO, c1, inp, dw1, db1, True, a1, ws, ws_bytes, config_id=cfg, stream=st)
        h.maxpool2x2(a1, 1, 16, 16, 32, p1, stream=st)
        h.conv2d(IM2COL, fc, p1, dw2, db2, False, y, ws, ws_bytes, config_id=cfg, splits=0, stream=st)

    net(dx, torch.cuda.current_stream())
    torch.cuda.synchronize()
    eager = y.cpu().numpy()
    ref1 = oc.conv2d(x, w1, b1, 1, 1, True)
    a1h = a1.cpu().numpy()
    assert np.all(np.abs(a1h - ref1) <= _tol(WINO, x, w1, b1, ref1, c1))
    p1h = oc.maxpool2x2(a1h)
    ref2 = oc.conv2d(p1h.reshape(1, 1, 1, -1), w2, b2, 1, 0, False)
    assert np.all(np.abs(eager - ref2) <= _tol(IM2COL, p1h, w2, b2, ref2, fc))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        net(dx, torch.cuda.current_stream())
    other = torch.from_numpy(_data(1, 16, 16, 8, 32, 3, 3, seed=93)[0]).cuda()
    for _ in range(3):
        net(other, torch.cuda.current_stream())     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), eager)


@pytest.mark.parametrize("case", [(1, 14, 14, 64, 128, 1), (2, 7, 9, 32, 48, 0)])
def test_winograd_pretransformed_filters(gpu, case):
    """Filters transformed once (kt_winograd_filter) and passed to the
    pre-transformed Winograd path give the same bits as the Winograd path
    that transforms them itself, within the oracle bound."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    n, H, W, C, O, pad = case
    cs = kt.conv_shape(n, H, W, C, O, 3, 3, 1, pad)
    x, w, b = _data(n, H, W, C, O, 3, 3, seed=950 + sum(case))
    cfg = h.configs().index((64, 64, 4, 16))
    plain = _run(h, torch, WINO, cs, x, w, b, True, cfg)
    dw = torch.from_numpy(w).cuda()
    U = torch.full((16 * C * O,), float("nan"), device="cuda")
    h.winograd_filter(dw, C, O, U)
    ws_bytes = kt.Handle.conv_workspace_bytes(cs, kt.CONV_WINOGRAD_PRETRANSFORMED)
    assert ws_bytes < kt.Handle.conv_workspace_bytes(cs, WINO)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    Ho, Wo = H + 2 * pad - 2, W + 2 * pad - 2
    dy = torch.full((n, Ho, Wo, O), float("nan"), device="cuda")
    h.conv2d(kt.CONV_WINOGRAD_PRETRANSFORMED, cs, torch.from_numpy(x).cuda(), U,
             torch.from_numpy(b).cuda(), True, dy, ws, ws_bytes, config_id=cfg)
    torch.cuda.synchronize()
    got = dy.cpu().numpy()
    assert np.array_equal(got, plain)
    ref = oc.conv2d(x, w, b, 1, pad, True)
    assert np.all(np.abs(got - ref) <= _tol(WINO, x, w, b, ref, cs))
