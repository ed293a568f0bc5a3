"""The split-K entry point that allocates nothing (kt_gemm_splitk_noalloc:
partial planes in the library's static device scratch) against
kt_gemm_splitk with a caller workspace.  Both run the same kernels on the
same slices, so the results must agree bit for bit; each is also held to
the FP32 bound against the FP64 oracle.  Two calls in a row, the second on
a smaller product (the scratch keeps the first call's planes), then an
automatic slice count, then a product too large for the scratch, which
must be refused before any launch."""
import math

import numpy as np
import pytest

import synth
from oracle import gemm as og

pytestmark = pytest.mark.gpu

F32 = 0


def _stored(x, trans):
    return np.ascontiguousarray(np.transpose(x, (0, 2, 1)) if trans else x)


def _run_both(h, torch, M, N, K, bt, ta, tb, splits, alpha, beta, cfg, seed):
    a = synth.uniform_operand(synth.operand_seed(seed, 0), bt * M * K).reshape(bt, M, K)
    b = synth.uniform_operand(synth.operand_seed(seed, 1), bt * K * N).reshape(bt, K, N)
    c0 = synth.uniform_operand(synth.operand_seed(seed, 2), bt * M * N).reshape(bt, M, N)
    dA = torch.from_numpy(_stored(a, ta)).cuda()
    dB = torch.from_numpy(_stored(b, tb)).cuda()
    ws_bytes = h.splitk_workspace_bytes(M, N, K, bt, splits)
    ws = torch.empty(max(ws_bytes, 4), dtype=torch.uint8, device="cuda")
    c_ws = torch.from_numpy(c0.copy()).cuda()
    c_na = torch.from_numpy(c0.copy()).cuda()
    used_ws = h.gemm_splitk(dA, dB, c_ws, splits, ws, ws_bytes, ta, tb, alpha, beta,
                            config_id=cfg)
    used_na = h.gemm_splitk_noalloc(dA, dB, c_na, splits, ta, tb, alpha, beta, config_id=cfg)
    torch.cuda.synchronize()
    got_ws, got_na = c_ws.cpu().numpy(), c_na.cpu().numpy()
    ref = og.gemm(M, N, K, bt, 0, 0, alpha, beta, a, K, M * K, b, N, K * N, c0, N, M * N)
    amax = np.abs(a).reshape(bt, -1).max(axis=1)
    bmax = np.abs(b).reshape(bt, -1).max(axis=1)
    tol = (1e-5 * math.sqrt(K) * abs(alpha) * amax * bmax)[:, None, None] \
        + 2.0 ** -23 * np.abs(beta * c0.astype(np.float64))
    return got_ws, got_na, ref, tol, used_ws, used_na


def test_noalloc_matches_workspace_entry_point(gpu):
    h, torch = gpu
    cfg = h.configs().index((64, 64, 4, 16))
    cases = [
        # (M, N, K, batch, transA, transB, splits, alpha, beta)
        (70, 300, 2500, 1, 0, 0, 8, 1.25, 0.5),   # 8 slices of 320, batched slice launch
        (33, 45, 1000, 2, 1, 1, 4, -0.75, 0.0),   # smaller, batched product, both transposed
    ]
    for i, (M, N, K, bt, ta, tb, sp, alpha, beta) in enumerate(cases):
        print(f"no-alloc split-K case {i}: {M}x{N}x{K} batch {bt} layout {ta}{tb} splits {sp}",
              flush=True)
        got_ws, got_na, ref, tol, u_ws, u_na = _run_both(h, torch, M, N, K, bt, ta, tb, sp,
                                                         alpha, beta, cfg, 8100 + i)
        assert u_ws == u_na and u_na > 1
        assert np.array_equal(got_ws.view(np.uint32), got_na.view(np.uint32))
        assert np.all(np.abs(got_na - ref) <= tol)


def test_noalloc_automatic_slices(gpu):
    h, torch = gpu
    cfg = h.configs().index((16, 64, 2, 32))
    print("no-alloc split-K automatic: 1x1000x4096", flush=True)
    got_ws, got_na, ref, tol, u_ws, u_na = _run_both(h, torch, 1, 1000, 4096, 1, 0, 0, 0, 1.0,
                                                     0.0, cfg, 8200)
    assert u_ws == u_na and u_na > 1
    assert np.array_equal(got_ws.view(np.uint32), got_na.view(np.uint32))
    assert np.all(np.abs(got_na - ref) <= tol)


def test_noalloc_refuses_products_beyond_the_scratch(gpu, kt):
    h, torch = gpu
    cap = h.splitk_noalloc_max_bytes()
    assert cap == 32 << 20
    M = N = 2048   # 4 slices x 2048 x 2048 floats = 64 MiB > 32 MiB
    dA = torch.zeros((1, M, 512), device="cuda")
    dB = torch.zeros((1, 512, N), device="cuda")
    dC = torch.zeros((1, M, N), device="cuda")
    with pytest.raises(kt.KtError) as e:
        h.gemm_splitk_noalloc(dA, dB, dC, 4, config_id=0)
    assert e.value.status == -5 and "static split-K scratch" in e.value.message
