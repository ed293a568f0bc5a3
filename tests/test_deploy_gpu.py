"""Deploy build (section 4 of the paper: only the pruned kernels ship in the
library): the library built from the recorded k-means choice contains only
those configurations, and each produces exactly the full build's bits."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_2008_13145_amd")
SPEC = os.path.join(PKG, "data", "deploy_f32.json")
DEPLOY = os.path.join(PKG, "libkt_deploy.so")


@pytest.fixture(scope="module")
def deploy(gpu):
    if not (os.path.exists(SPEC) and os.path.exists(DEPLOY)):
        pytest.skip("no deploy choice recorded / deploy library not built")
    import paper_2008_13145_amd as kt
    spec = json.load(open(SPEC))
    hd = kt.Handle(0, libpath=DEPLOY)
    yield spec, hd
    hd.close()


def _config_ids(spec):
    """Configurations the deploy build holds: those of the chosen kernels (a
    split-K variant runs its base configuration's code)."""
    return set(spec.get("config_ids", spec["chosen"]))


def test_only_chosen_configs_compiled(deploy, kt):
    spec, hd = deploy
    chosen = set(spec["chosen"])
    assert len(chosen) == spec["k"]
    cfg_ids = _config_ids(spec)
    assert cfg_ids == {hd.get_kernel(c)[1] for c in chosen}
    for cid in range(hd.num_configs()):
        for ta, tb in synth.LAYOUTS:
            assert hd.config_compiled(cid, ta, tb) == (cid in cfg_ids)
    if "kernels" in spec:
        assert [list(hd.get_kernel(c)[0]) for c in spec["chosen"]] == spec["kernels"]
    # every split-K variant of a kept configuration is available, no other
    for v in range(hd.num_configs(), hd.num_kernels()):
        assert hd.config_compiled(v, 0, 0) == (hd.get_kernel(v)[1] in cfg_ids)
    assert os.path.getsize(DEPLOY) < os.path.getsize(kt.LIB_PATH)


def test_deploy_matches_full_build_bitwise(deploy, gpu):
    spec, hd = deploy
    h, torch = gpu
    M, N, K, bt = 201, 333, 157, 2
    for ta, tb in synth.LAYOUTS:
        a = synth.uniform_operand(11 + ta, bt * M * K).reshape(bt, K, M) if ta else \
            synth.uniform_operand(11, bt * M * K).reshape(bt, M, K)
        b = synth.uniform_operand(12 + tb, bt * K * N).reshape(bt, N, K) if tb else \
            synth.uniform_operand(12, bt * K * N).reshape(bt, K, N)
        dA, dB = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        for cid in spec["chosen"]:
            c1 = torch.zeros((bt, M, N), dtype=torch.float32, device="cuda")
            c2 = torch.zeros((bt, M, N), dtype=torch.float32, device="cuda")
            h.gemm(dA, dB, c1, ta, tb, 1.0, 0.0, config_id=cid)
            hd.gemm(dA, dB, c2, ta, tb, 1.0, 0.0, config_id=cid)
            torch.cuda.synchronize()
            assert torch.equal(c1, c2)


def test_deploy_rejects_pruned_config_and_selects(deploy, gpu):
    import paper_2008_13145_amd as kt
    spec, hd = deploy
    h, torch = gpu
    other = next(c for c in range(hd.num_configs()) if c not in _config_ids(spec))
    d = torch.zeros(64 * 64, dtype=torch.float32, device="cuda")
    st = hd.gemm_raw(kt.F32, kt.shape(8, 8, 8), 1.0, d, 8, 0, d, 8, 0, 0.0, d, 8, 0,
                     config_id=other, check=False)
    assert st == -2
    # a selector fitted over the deployed set picks only deployed kernels
    problems = synth.sweep_problems(40, 31)
    rng = np.random.default_rng(0)
    T = rng.integers(1000, 100000, size=(len(problems), hd.num_kernels())).astype(np.int64)
    hd.fit_selector(kt.SEL_DT_A, problems, T, spec["chosen"])
    for p in problems[:20]:
        assert hd.select(*p) in spec["chosen"]
