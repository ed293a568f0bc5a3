#!/usr/bin/env python3
"""Benchmark of the deployed, pruned and selected FP32 GEMM library on MI355X.

Workload (one "step"): the 1200 GEMM problems of the sweep set -- 300 seeded
log-uniform (M, N, K, batch) shapes, M, N, K in 16..4096 and batch in 1..64,
each in the four transpose layouts -- run once each through the library's
deployed path: kt_gemm with config_id = -1, so the fitted selector (a
decision tree over the k kernels chosen by k-means pruning of the benchmark
table) picks the configuration and the chosen kernel is launched.  Operands
live in HBM before timing starts.

Setup (untimed, reported): the benchmark table of every configuration on
every problem (the sweep, sections 3 and 3.1 of the paper) is loaded from
the committed dataset; k-means pruning runs on the GPU over the training
problems (section 4); the decision trees A/B/C and the MLP cost model are
fitted on the training problems (section 5.1) and evaluated on the held-out
test problems against exhaustive search (section 4.3).

Prints one JSON line.  Only one GPU is supported: --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
SEL_NAMES = {0: "DT-A", 1: "DT-B", 2: "DT-C", 3: "MLP"}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _geomean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(math.exp(np.mean(np.log(x))))


def cpu_baseline(problems, budget_s=15.0, seed=13145, tuning=None):
    """The FP64 CPU oracle (test infrastructure) timed on a bounded, seeded
    sample of the same problem set: problems are taken in a fixed seeded order
    (those up to 2 GFLOP each) until the time budget is spent."""
    import synth
    from oracle import gemm as og
    rng = np.random.default_rng(seed)
    small = [p for p in problems if 2 * p[0] * p[1] * p[2] * p[3] <= 2e9]
    order = rng.permutation(len(small))
    flops, t_tot, n = 0.0, 0.0, 0
    for i in order:
        M, N, K, b, ta, tb = small[i]
        a = synth.uniform_operand(synth.operand_seed(n, 0), b * M * K)
        bb = synth.uniform_operand(synth.operand_seed(n, 1), b * K * N)
        lda = M if ta else K
        ldb = K if tb else N
        t0 = time.perf_counter()
        og.gemm(M, N, K, b, ta, tb, 1.0, 0.0, a, lda, M * K, bb, ldb, K * N)
        t_tot += time.perf_counter() - t0
        flops += 2.0 * M * N * K * b
        n += 1
        if t_tot >= budget_s:
            break
    # the single 256^3 GEMM workload, on one core and on all of them
    n_all = og.max_threads()
    a = synth.uniform_operand(synth.operand_seed(synth.SEED + 1, 0), 256 * 256)
    bb = synth.uniform_operand(synth.operand_seed(synth.SEED + 1, 1), 256 * 256)
    single = {}
    for nt in (1, n_all):
        og.set_threads(nt)
        t0 = time.perf_counter()
        og.gemm(256, 256, 256, 1, 0, 0, 1.0, 0.0, a, 256, 65536, bb, 256, 65536)
        single[f"{nt}_core" + ("s" if nt > 1 else "")] = round((time.perf_counter() - t0) * 1e3, 3)
    og.set_threads(n_all)
    tuning_s = None
    if tuning is not None:
        # the tuning oracles on the deployed pruning's inputs (training rows
        # of the measured table, its normalization, k): normalization plus
        # 10-restart k-means, and decision tree B's fit
        from oracle import cart, kmeans as okm, normalize as onorm
        T_tr, shapes_tr, norm, k = tuning
        t0 = time.perf_counter()
        X = onorm.normalize(T_tr, norm)
        km = okm.kmeans(X, k, okm.restart_draws(synth.SplitMix64, synth.SEED, 10, k), 300)
        t1 = time.perf_counter()
        ch = okm.centroids_to_configs(km["centroids"])
        md, ml = cart.TREE_PARAMS["B"]
        cart.fit(np.array(shapes_tr, dtype=np.int64), cart.labels_from_times(T_tr, ch), k, md, ml)
        t2 = time.perf_counter()
        tuning_s = {"prune_s": round(t1 - t0, 3), "fit_dt_b_s": round(t2 - t1, 4)}
    return dict(value=round(flops / t_tot / 1e12, 6), unit="TFLOP/s", cores=n_all,
                kind="oracle",
                sample=f"{n} problems of the 1200-problem set (seeded order, each <= 2 GFLOP), "
                       f"{flops / 1e9:.1f} GFLOP in {t_tot:.1f} s, FP64 triple loop",
                single_gemm_256_ms=single, tuning=tuning_s)


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from a committed rocprofv3 counter
    summary (profiles/*_traffic.txt), if one exists for this kernel and the
    kernel source has not changed since the counters were taken; else None."""
    import glob
    import hashlib
    hdr = "gemm_f32_dma.hpp" if kernel_name.startswith("gemm_f32_dma_kernel") else "gemm_f32.hpp"
    src = os.path.join(ROOT, "paper_2008_13145_amd", "csrc", hdr)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt"))):
        fields = {}
        for line in open(path):
            if "=" in line and not line.startswith(" "):
                key, _, val = line.partition("=")
                fields[key.strip()] = val.strip()
        if fields.get("kernel") == kernel_name and fields.get("kernel_source_sha256", "").split()[:1] == [sha]:
            return int(fields["traffic_bytes_per_launch"])
    return None


def single_gemm_section(kt, h, torch, synth, stream, reps=200, warm=10):
    """The single FP32 GEMM workload: M = N = K = 256, batch 1, NN, alpha 1,
    beta 0, operands from seed SEED + 1, one fixed configuration (64x64 work
    group, 4x4 thread tile, K-tile 16).  Mean over `reps` launches after
    `warm` warm-ups, and the same launches replayed from one captured graph
    (its parity is a GPU test; the oracle's time is in cpu_baseline)."""
    M = N = K = 256
    cid = h.configs().index((64, 64, 4, 16))
    a = synth.uniform_operand(synth.operand_seed(synth.SEED + 1, 0), M * K).reshape(1, M, K)
    b = synth.uniform_operand(synth.operand_seed(synth.SEED + 1, 1), K * N).reshape(1, K, N)
    dA = torch.from_numpy(a).cuda()
    dB = torch.from_numpy(b).cuda()
    dC = torch.empty((1, M, N), dtype=torch.float32, device="cuda")
    shp = kt.shape(M, N, K)

    def launch(st):
        h.gemm_raw(kt.F32, shp, 1.0, dA, K, M * K, dB, N, K * N, 0.0, dC, N, M * N,
                   config_id=cid, stream=st)
    for _ in range(warm):
        launch(stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cs = torch.cuda.current_stream()
        for _ in range(reps):
            launch(cs)
    g.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    us_graph = e0.elapsed_time(e1) * 1e3 / reps
    F = 2.0 * M * N * K
    t_roof_us = max(F / (FP32_PEAK_TFLOPS * 1e12), 4.0 * (M * K + K * N + M * N) / 8e12) * 1e6
    return {"config": [64, 64, 4, 16], "us_per_launch": round(us, 3),
            "tflops": round(F / (us * 1e-6) / 1e12, 3),
            "us_per_launch_graph": round(us_graph, 3),
            "tflops_graph": round(F / (us_graph * 1e-6) / 1e12, 3),
            "pct_mfma_peak_graph": round(100 * F / (us_graph * 1e-6) / 1e12 / FP32_PEAK_TFLOPS, 2),
            "t_roof_us": round(t_roof_us, 4), "frac_of_t_roof_graph": round(t_roof_us / us_graph, 4),
            "work_groups": (M // 64) * (N // 64)}


def splitk_section(kt, h, torch, T, problems, plans, chosen, stream, reps=5):
    """Split-K on the rows whose exhaustive-best configuration leaves the chip
    under-filled (fewer than 256 work-groups) with K >= 512: each row's
    exhaustive-best plain launch against the best split-K launch over splits
    {2, 4, 8, 16} x (that configuration and the k deployed ones), both timed
    live on resident operands (mean of `reps` launches after one warm-up)."""
    cfgs = h.configs()
    n_plain = len(cfgs)
    Tp = T[:, :n_plain]          # the configurations' columns (split-K variants are timed here)
    rows = []
    for r, (M, N, K, bt, ta, tb) in enumerate(problems):
        bm, bn = cfgs[int(np.argmin(Tp[r]))][:2]
        if K >= 512 and -(-M // bm) * -(-N // bn) * bt < 256:
            rows.append(r)
    if not rows:
        return None
    ws_bytes = max(kt.Handle.splitk_workspace_bytes(*problems[r][:4], 16) for r in rows)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    t_plain, t_split, best_pick = [], [], []
    for r in rows:
        pl = plans[r]
        best = int(np.argmin(Tp[r]))
        t_plain.append(timed(lambda: h.gemm_raw(kt.F32, pl[0], 1.0, pl[1], pl[2], pl[3], pl[4],
                                                pl[5], pl[6], 0.0, pl[7], pl[8], pl[9],
                                                config_id=best, stream=stream)))
        cand = []
        for cid in dict.fromkeys([best] + [h.get_kernel(c)[1] for c in chosen]):
            for sp in (2, 4, 8, 16):
                us = timed(lambda: h.gemm_splitk_raw(kt.F32, pl[0], sp, 1.0, pl[1], pl[2], pl[3],
                                                     pl[4], pl[5], pl[6], 0.0, pl[7], pl[8],
                                                     pl[9], ws, ws_bytes, config_id=cid,
                                                     stream=stream))
                cand.append((us, sp, cid))
        us, sp, cid = min(cand)
        t_split.append(us)
        best_pick.append((sp, cid))
    t_plain, t_split = np.array(t_plain), np.array(t_split)
    speed = t_plain / np.minimum(t_plain, t_split)
    i = int(np.argmax(t_plain / t_split))
    return {"rows": len(rows), "rows_where_split_k_wins": int((t_split < t_plain).sum()),
            "geomean_speedup_best_of_both": round(_geomean(speed), 4),
            "max_speedup": round(float(t_plain[i] / t_split[i]), 3),
            "max_speedup_problem": list(problems[rows[i]]),
            "max_speedup_pick": {"splits": best_pick[i][0], "config": list(cfgs[best_pick[i][1]])},
            "us_plain_sum": round(float(t_plain.sum()), 1),
            "us_best_of_both_sum": round(float(np.minimum(t_plain, t_split).sum()), 1)}


# VGG16 (configuration D of Simonyan and Zisserman): 3x3 convolutions with
# stride 1 and padding 1 (output channels listed), "M" = 2x2 max pool, then
# three fully connected layers.
VGG16_CONV = [64, 64, "M", 128, 128, "M", 256, 256, 256, "M", 512, 512, 512, "M",
              512, 512, 512, "M"]
VGG16_FC = [(7 * 7 * 512, 4096), (4096, 4096), (4096, 1000)]


def vgg16_section(kt, h, torch, synth, stream, reps=10, cfg_reps=3):
    """Single-image VGG16 inference (224x224x3, random weights scaled by
    1/sqrt(fan-in), FP32, NHWC): 13 3x3 convolutions with ReLU, 5 max pools,
    3 fully connected layers run as 1x1 convolutions of a 1x1 image.

    The selector's inference takes no timing: a fixed lowering rule (Winograd
    with filters transformed at load for the 3x3 stride-1 layers, im2col for
    the rest) and the deployed selector's kernel for every GEMM (config -1;
    a selected split-K kernel runs split -- the fully connected layers, M = 1,
    lie outside the training shapes and go to the fallback, which times the
    chosen kernels and their split-K variants once; the same inference with
    the exhaustive fallback, every kernel of the library timed once per
    out-of-range shape, is reported beside it).  The exhaustive
    reference takes, per layer, the fastest of every lowering x every
    configuration (x split counts 2..32 for the fully connected layers).
    Also reported: the best lowering per layer among the selector's options
    chosen by timing them (labelled as such)."""
    layers = []   # (kind, conv_shape)
    H, C = 224, 3
    for v in VGG16_CONV:
        if v == "M":
            layers.append(("pool", (H, C)))
            H //= 2
        else:
            layers.append(("conv", kt.conv_shape(1, H, H, C, v)))
            C = v
    for (fi, fo) in VGG16_FC:
        layers.append(("fc", kt.conv_shape(1, 1, 1, fi, fo, 1, 1, 1, 0)))
    convs = [cs for kind, cs in layers if kind != "pool"]
    ws_bytes = max(max(kt.Handle.conv_workspace_bytes(cs, kt.CONV_IM2COL, sp) for sp in (0, 1, 32))
                   for cs in convs)
    ws_bytes = max([ws_bytes] + [kt.Handle.conv_workspace_bytes(cs, kt.CONV_WINOGRAD)
                                 for cs in convs if cs.R == 3])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    weights, biases = [], []
    for i, cs in enumerate(convs):
        n_w = cs.R * cs.S * cs.Cin * cs.Cout
        wt = torch.empty(n_w, dtype=torch.float32, device="cuda")
        h.fill_uniform(wt, n_w, synth.operand_seed(synth.SEED + 100 + i, 1), stream=stream)
        wt.mul_(1.0 / math.sqrt(cs.R * cs.S * cs.Cin))
        bt = torch.empty(cs.Cout, dtype=torch.float32, device="cuda")
        h.fill_uniform(bt, cs.Cout, synth.operand_seed(synth.SEED + 100 + i, 2), stream=stream)
        weights.append(wt)
        biases.append(bt)
    # Winograd filters transformed once, when the weights are loaded
    wino_u = {}
    for i, cs in enumerate(convs):
        if cs.R == 3:
            wino_u[i] = torch.empty(16 * cs.Cin * cs.Cout, dtype=torch.float32, device="cuda")
            h.winograd_filter(weights[i], cs.Cin, cs.Cout, wino_u[i], stream=stream)

    def wt_of(li, algo):
        return wino_u[li] if algo == kt.CONV_WINOGRAD_PRETRANSFORMED else weights[li]
    x0 = torch.empty(224 * 224 * 3, dtype=torch.float32, device="cuda")
    h.fill_uniform(x0, x0.numel(), synth.operand_seed(synth.SEED + 99, 0), stream=stream)
    buf = [torch.empty(224 * 224 * 64, dtype=torch.float32, device="cuda") for _ in range(2)]
    flops = sum(2.0 * cs.H * cs.W * cs.Cout * cs.R * cs.S * cs.Cin for cs in convs)
    last = len(convs) - 1

    def forward(choice, st=stream):
        """choice[li] = (algo, config_id, splits)."""
        src, li = x0, 0
        for kind, cs in layers:
            dst = buf[0] if src is not buf[0] else buf[1]
            if kind == "pool":
                Hp, Cp = cs
                h.maxpool2x2(src, 1, Hp, Hp, Cp, dst, stream=st)
            else:
                algo, cid, sp = choice[li]
                h.conv2d(algo, cs, src, wt_of(li, algo), biases[li], li < last, dst, ws, ws_bytes,
                         config_id=cid, splits=sp, stream=st)
                li += 1
            src = dst
        return src

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        fn()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    cfgs = h.configs()
    per, sel_choice, ex_choice, rule_choice = [], [], [], []
    for li, cs in enumerate(convs):
        xin = torch.empty(cs.H * cs.W * cs.Cin, dtype=torch.float32, device="cuda")
        h.fill_uniform(xin, xin.numel(), synth.operand_seed(synth.SEED + 200 + li, 0), stream=stream)
        out = torch.empty(cs.H * cs.W * cs.Cout, dtype=torch.float32, device="cuda")

        def run(algo, cid, sp):
            return timed(lambda: h.conv2d(algo, cs, xin, wt_of(li, algo), biases[li], True, out, ws,
                                          ws_bytes, config_id=cid, splits=sp, stream=stream), cfg_reps)
        row = {"layer": li, "H": cs.H, "Cin": cs.Cin, "Cout": cs.Cout, "R": cs.R}
        sel_opts, ex_opts = [], []
        lowerings = [(kt.CONV_IM2COL, "im2col")] + ([(kt.CONV_WINOGRAD, "winograd")] if cs.R == 3 else [])
        for algo, name in lowerings:
            t_sel = timed(lambda: h.conv2d(algo, cs, xin, weights[li], biases[li], True, out, ws,
                                           ws_bytes, stream=stream), reps)
            sel_opts.append((t_sel, (algo, -1, 1)))
            ent = {"ms_selected": round(t_sel, 4)}
            if algo == kt.CONV_IM2COL:
                t_auto = timed(lambda: h.conv2d(algo, cs, xin, weights[li], biases[li], True, out,
                                                ws, ws_bytes, splits=0, stream=stream), reps)
                sel_opts.append((t_auto, (algo, -1, 0)))
                ent["ms_selected_auto_split"] = round(t_auto, 4)
            split_set = (1, 2, 4, 8, 16, 32) if (algo == kt.CONV_IM2COL and cs.H == 1) else (1,)
            best = min((run(algo, c, sp), (algo, c, sp)) for sp in split_set for c in range(len(cfgs)))
            ex_opts.append(best)
            ent.update({"ms_exhaustive": round(best[0], 4), "exhaustive_config": list(cfgs[best[1][1]]),
                        "exhaustive_splits": best[1][2],
                        "gemm": list(kt.Handle.conv_gemm_shape(cs, algo)[:4])})
            row[name] = ent
            if algo == kt.CONV_WINOGRAD:   # the same layer with filters transformed at load time
                pre = kt.CONV_WINOGRAD_PRETRANSFORMED
                t_pre = timed(lambda: h.conv2d(pre, cs, xin, wino_u[li], biases[li], True, out, ws,
                                               ws_bytes, stream=stream), reps)
                sel_opts.append((t_pre, (pre, -1, 1)))
                ex_opts.append((run(pre, best[1][1], 1), (pre, best[1][1], 1)))
                row["winograd_pretransformed"] = {"ms_selected": round(t_pre, 4)}
        sel_choice.append(min(sel_opts)[1])
        ex_choice.append(min(ex_opts)[1])
        # the selector's pick for this layer's GEMM under the lowering rule
        algo_r = kt.CONV_WINOGRAD_PRETRANSFORMED if (cs.R == 3 and cs.stride == 1) else kt.CONV_IM2COL
        g_shape = kt.Handle.conv_gemm_shape(cs, kt.CONV_WINOGRAD if algo_r != kt.CONV_IM2COL else algo_r)
        pick = h.select(*g_shape)
        row["rule"] = {"lowering": "winograd_pretransformed" if algo_r != kt.CONV_IM2COL else "im2col",
                       "selected_kernel": list(h.get_kernel(pick)[0]),
                       "ms": round(timed(lambda: h.conv2d(algo_r, cs, xin, wt_of(li, algo_r), biases[li],
                                                          True, out, ws, ws_bytes, stream=stream),
                                         reps), 4)}
        box = h.selector_info()
        if any(not (box["box_lo"][f] <= g_shape[f] <= box["box_hi"][f]) for f in range(4)):
            # outside the training shapes: the exhaustive fallback instead
            h.set_fallback(2)
            pick2 = h.select(*g_shape)
            row["rule_exhaustive_fallback"] = {
                "selected_kernel": list(h.get_kernel(pick2)[0]),
                "ms": round(timed(lambda: h.conv2d(algo_r, cs, xin, wt_of(li, algo_r), biases[li],
                                                   True, out, ws, ws_bytes, stream=stream), reps), 4)}
            h.set_fallback(1)
        rule_choice.append((algo_r, -1, 1))
        per.append(row)
    ms = {
        "selector": timed(lambda: forward(rule_choice), reps),
        "exhaustive": timed(lambda: forward(ex_choice), reps),
        "im2col_selector": timed(lambda: forward([(kt.CONV_IM2COL, -1, 1)] * len(convs)), reps),
        "winograd_selector": timed(lambda: forward([(kt.CONV_WINOGRAD if cs.R == 3 else kt.CONV_IM2COL,
                                                     -1, 1) for cs in convs]), reps),
        "timed_lowering_selector_kernels": timed(lambda: forward(sel_choice), reps),
    }
    h.set_fallback(2)
    ms["selector_exhaustive_fallback"] = timed(lambda: forward(rule_choice), reps)
    h.set_fallback(1)
    # the selector's inference captured once in a graph and replayed
    out_eager = forward(rule_choice).clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out_buf = forward(rule_choice, torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(out_buf, out_eager))
    ms["selector_graph"] = timed(g.replay, reps)
    torch.cuda.synchronize()
    names = {kt.CONV_IM2COL: "im2col", kt.CONV_WINOGRAD: "winograd",
             kt.CONV_WINOGRAD_PRETRANSFORMED: "winograd_pretransformed"}
    fc = [r for r in per if r["H"] == 1]
    return {"ms_per_inference": {kk: round(v, 4) for kk, v in ms.items()},
            "gflop_direct": round(flops / 1e9, 2),
            "tflops_effective_selector": round(flops / (ms["selector"] * 1e-3) / 1e12, 2),
            "selector_pct_of_exhaustive": round(100 * ms["exhaustive"] / ms["selector"], 2),
            "fc1_selector_vs_exhaustive": round(fc[0]["rule"]["ms"] / fc[0]["im2col"]["ms_exhaustive"], 3),
            "fc1_selector_exhaustive_fallback_vs_exhaustive": round(
                fc[0]["rule_exhaustive_fallback"]["ms"] / fc[0]["im2col"]["ms_exhaustive"], 3)
            if "rule_exhaustive_fallback" in fc[0] else None,
            "exhaustive_choice": [[names[a], list(cfgs[c]), sp] for a, c, sp in ex_choice],
            "timed_lowering_choice": [[names[a], sp] for a, _, sp in sel_choice],
            "graph_replay_matches_eager": graph_ok,
            "layers": per}


def repeatability(kt, h, torch, T, problems, plans, stream, n_rows=50, rounds=5, seed=13145):
    """Re-time the best kernel of `n_rows` seeded rows `rounds` times with the
    sweep's protocol (operands resident, two warm-up launches, then launches
    worth about 5 ms per timing, at least 3, at most 200): coefficient of
    variation of the per-launch time across rounds, and the ratio of the
    re-timed mean to the table's entry."""
    rng = np.random.default_rng(seed)
    rows = sorted(int(r) for r in rng.choice(len(problems), n_rows, replace=False))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    cvs, ratios = [], []
    for r in rows:
        best = int(np.argmin(T[r]))
        pl = plans[r]
        t_tab = float(T[r, best]) * 1e-6              # ms

        def launch():
            h.gemm_raw(kt.F32, pl[0], 1.0, pl[1], pl[2], pl[3], pl[4], pl[5], pl[6], 0.0,
                       pl[7], pl[8], pl[9], config_id=best, stream=stream)
        n = int(min(200, max(3, np.ceil(5.0 / max(t_tab, 1e-4)))))
        ts = []
        for _ in range(rounds):
            for _ in range(2):
                launch()
            e0.record(stream)
            for _ in range(n):
                launch()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / n)
        ts = np.array(ts)
        cvs.append(float(ts.std() / ts.mean()))
        ratios.append(float(ts.mean() / t_tab))
    cvs, ratios = np.array(cvs), np.array(ratios)
    return {"rows": n_rows, "rounds": rounds, "cv_median": round(float(np.median(cvs)), 4),
            "cv_p90": round(float(np.percentile(cvs, 90)), 4), "cv_max": round(float(cvs.max()), 4),
            "retimed_over_table_median": round(float(np.median(ratios)), 4),
            "retimed_over_table_p10_p90": [round(float(np.percentile(ratios, 10)), 4),
                                           round(float(np.percentile(ratios, 90)), 4)]}


def gpu_state():
    """Clocks, power and temperature of the GPU from rocm-smi (a child
    process; None if it is unavailable)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--showtemp", "--json"],
                           capture_output=True, text=True, timeout=30)
        card = next(iter(json.loads(r.stdout).values()))
    except Exception:
        return None
    keep = ("sclk", "mclk", "fclk", "power", "temperature")
    return {k: v for k, v in card.items() if any(w in k.lower() for w in keep)}


def deploy_info(chosen, n_configs):
    """Size of the pruned deploy build (section 4: only the k chosen kernels
    ship) against the full build, and whether its recorded choice is the one
    this run made."""
    import json as _json
    pkg = os.path.join(ROOT, "paper_2008_13145_amd")
    full = os.path.join(pkg, "libkt.so")
    dep = os.path.join(pkg, "libkt_deploy.so")
    spec_path = os.path.join(pkg, "data", "deploy_f32.json")
    out = {"full_library_bytes": os.path.getsize(full) if os.path.exists(full) else None,
           "full_kernels": "%d FP32 + %d BF16 + %d FP8 configurations x 4 layouts" % tuple(n_configs)}
    if os.path.exists(dep) and os.path.exists(spec_path):
        spec = _json.load(open(spec_path))
        out.update({"deploy_library_bytes": os.path.getsize(dep),
                    "deploy_kernels": f"{len(spec['chosen'])} FP32 kernels ({len(spec['config_ids'])} "
                                      "configurations x 4 layouts, split-K variants of them included)",
                    "deploy_choice_matches_this_run": [int(c) for c in spec["chosen"]] == [int(c) for c in chosen]})
    return out


def _grouped_layout(kt, h, torch, synth, shapes, stream, padded):
    """Device operands of the grouped workload: BF16 A (M x lda) and B
    (K x ldb) converted on the GPU from one seeded FP32 stream, FP32 C.
    padded: rows padded to a multiple of 8 elements (16 bytes, allocated in
    full); else dense rows.  Returns pointers, leading dimensions and the FP32
    source of each member's values (for the error report)."""
    a256 = lambda v: (v + 255) // 256 * 256
    rnd = (lambda v: (v + 7) // 8 * 8) if padded else (lambda v: v)
    offs_a, offs_b, offs_c, ld = [], [], [], []
    na = nb = nc = 0
    for (M, N, K) in shapes:
        lda, ldb = rnd(K), rnd(N)
        ld.append((lda, ldb, N))
        offs_a.append(na); na += a256(M * lda * 2)
        offs_b.append(nb); nb += a256(K * ldb * 2)
        offs_c.append(nc); nc += a256(M * N * 4)
    src = torch.empty((max(na, nb) + 3) // 2, dtype=torch.float32, device="cuda")
    h.fill_uniform(src, src.numel(), synth.operand_seed(synth.SEED + 4, 0), stream=stream)
    pa = torch.empty(na, dtype=torch.uint8, device="cuda")
    pb = torch.empty(nb, dtype=torch.uint8, device="cuda")
    pc = torch.empty(nc, dtype=torch.uint8, device="cuda")
    h.convert_bf16(src, na // 2, pa, stream=stream)
    h.convert_bf16(src, nb // 2, pb, stream=stream)
    return dict(A=[pa.data_ptr() + o for o in offs_a], B=[pb.data_ptr() + o for o in offs_b],
                C=[pc.data_ptr() + o for o in offs_c], ld=ld, src=src, offs_a=offs_a,
                offs_b=offs_b, offs_c=offs_c, bufs=(pa, pb, pc))


def grouped_section(kt, h, torch, synth, stream, reps=20):
    """The persistent grouped BF16 GEMM on its workload (512 uneven GEMMs,
    M, N, K log-uniform in 32..2048, A M x K, B K x N, FP32 out): the
    library's autotuner picks (tile pair, small-member area, schedule, order,
    work-groups per CU) on the real group, then one hipGraph launch runs every
    member.  Two storage layouts: rows padded to 16 bytes (the DMA pipeline)
    and dense rows.  Reported against the sum over members of each one's
    roofline time at peak BF16 MFMA rate and HBM bandwidth, and against one
    kt_gemm launch per member with the configuration the BF16 selector picks
    for it (the same storage, whole rows promised)."""
    shapes = synth.grouped_shapes()
    flops = sum(2.0 * m * n * k for (m, n, k) in shapes)
    roof_ms = sum(max(2.0 * m * n * k / 2.5e15, (2.0 * (m * k + k * n) + 4.0 * m * n) / 8e12)
                  for (m, n, k) in shapes) * 1e3
    wsb = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for (m, n, k) in shapes])
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {"members": len(shapes), "gflop": round(flops / 1e9, 2),
           "sum_member_roofline_ms": round(roof_ms, 4)}
    for name, padded in (("rows_padded_16B", True), ("dense_rows", False)):
        L = _grouped_layout(kt, h, torch, synth, shapes, stream, padded)
        A, B, C, ld = L["A"], L["B"], L["C"], L["ld"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, best_ms, evals = h.autotune_grouped(shapes, A, B, C, ws, wsb, stream=stream, ld=ld)
        tune_s = time.perf_counter() - t0
        plan = h.grouped_plan(shapes, A, B, C, workspace=ws, ws_bytes=wsb, stream=stream, ld=ld)
        n_work = h.grouped_info(plan)[0]
        for _ in range(3):
            h.grouped_launch(plan, stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            h.grouped_launch(plan, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # one launch per member: the selector's pick (when a BF16 selector is
        # fitted) and the grouped plan's large tile
        h.set_full_rows(padded)
        sel_ms = None
        if h.selector_info(kt.BF16)["kind"] >= 0:
            picks = [h.select(M, N, K, dtype=kt.BF16) for (M, N, K) in shapes]

            def run_selected():
                for i, (M, N, K) in enumerate(shapes):
                    h.gemm_raw(kt.BF16, kt.shape(M, N, K), 1.0, A[i], ld[i][0], 0, B[i], ld[i][1], 0,
                               0.0, C[i], N, 0, config_id=picks[i], stream=stream)
            run_selected()
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(3):
                run_selected()
            e1.record(stream)
            torch.cuda.synchronize()
            sel_ms = e0.elapsed_time(e1) / 3
        e0.record(stream)
        for i, (M, N, K) in enumerate(shapes):
            h.gemm_raw(kt.BF16, kt.shape(M, N, K), 1.0, A[i], ld[i][0], 0, B[i], ld[i][1], 0, 0.0,
                       C[i], N, 0, config_id=best[0], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        same_ms = e0.elapsed_time(e1)
        h.set_full_rows(False)
        # per-member relative Frobenius error of the graph launch's output
        # against the product of the original FP32 operands in FP64 (computed
        # on the GPU here; the parity tests hold each member to 1e-2 against
        # the CPU oracle)
        h.grouped_launch(plan, stream=stream)
        torch.cuda.synchronize()
        errs = []
        src, pc = L["src"], L["bufs"][2]
        for i, (M, N, K) in enumerate(shapes):
            lda, ldb, _ = ld[i]
            oa, ob = L["offs_a"][i] // 2, L["offs_b"][i] // 2
            a64 = src[oa: oa + M * lda].view(M, lda)[:, :K].double()
            b64 = src[ob: ob + K * ldb].view(K, ldb)[:, :N].double()
            ref = a64 @ b64
            c = pc[L["offs_c"][i]: L["offs_c"][i] + M * N * 4].view(torch.float32).view(M, N).double()
            errs.append(float(torch.linalg.norm(c - ref) / torch.linalg.norm(ref)))
        errs = np.array(errs)
        h.grouped_destroy(plan)
        bm, bn, tt, bk = h.get_config(best[0], kt.BF16)
        out[name] = {
            "tile": [bm, bn, tt, bk],
            "small_tile": list(h.get_config(best[1], kt.BF16)) if best[1] >= 0 else None,
            "small_max_area": best[2], "schedule": best[3], "order": best[4],
            "wgs_per_cu": best[5], "pipeline": "register-staged" if best[6] else "LDS DMA where the rows allow",
            "work_items": n_work,
            "autotune_evaluations": evals, "autotune_s": round(tune_s, 3),
            "ms_per_launch": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "roofline": {"bound": "per-member max(MFMA at 2.5 PF/s, HBM at 8 TB/s), summed",
                         "achieved_ms": round(ms, 4), "roofline_ms": round(roof_ms, 4),
                         "frac": round(roof_ms / ms, 4)},
            "member_rel_frobenius_error": {
                "max": float(f"{errs.max():.3e}"), "median": float(f"{np.median(errs):.3e}"),
                "p90": float(f"{np.percentile(errs, 90):.3e}"), "bound": 1e-2,
                "members_within_bound": int((errs <= 1e-2).sum())},
            "separate_launches_selected_ms": None if sel_ms is None else round(sel_ms, 3),
            "speedup_vs_separate_selected": None if sel_ms is None else round(sel_ms / ms, 2),
            "separate_launches_same_tile_ms": round(same_ms, 3),
            "speedup_vs_separate_same_tile": round(same_ms / ms, 2)}
        del L
    return out


def selection_latency(kt, h, torch, problems, stream, reps=20):
    """Cost of a selection with the handle's current selector: host
    kt_select per call, and the device batch selection (kt_select_batch) for
    one shape and for all of them, timed with HIP events on the launch
    stream."""
    arr = np.array([[m, n, k, b, (ta | (tb << 32))] for (m, n, k, b, ta, tb) in problems], np.int64)
    d_shapes = torch.from_numpy(arr).cuda()
    d_ids = torch.zeros(len(problems), dtype=torch.int32, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {}
    for n in (1, len(problems)):
        h.select_batch(d_shapes, n, d_ids, stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            h.select_batch(d_shapes, n, d_ids, stream=stream)
        e1.record(stream)
        e1.synchronize()
        out[f"device_batch_{n}_us"] = round(e0.elapsed_time(e1) * 1e3 / reps, 3)
    t0 = time.perf_counter()
    for _ in range(3):
        for p in problems:
            h.select(*p)
    out["host_us_per_shape"] = round((time.perf_counter() - t0) / (3 * len(problems)) * 1e6, 3)
    out["selector"] = {0: "DT-A", 1: "DT-B", 2: "DT-C", 3: "MLP"}.get(h.selector_info()["kind"])
    return out


def lowp_section(kt, h, torch, tune, synth, problems, T32, pool, plans, flops, k, steps, stream,
                 mws, mws_bytes, pad=False):
    """BF16 / FP8 paths on the same 1200 problems: their own sweep tables,
    k-means pruning on the training shapes, decision trees A/B/C and the MLP
    scored on the held-out shapes, the selector chosen on validation shapes
    deployed for a live pass (HIP events around every launch, on the launch
    stream), the dominant kernel against its MFMA peak, and the speedup over
    the FP32 exhaustive best."""
    out = {}
    train, test = synth.train_test_split()
    tr_rows, te_rows = synth.rows_of_shapes(train), synth.rows_of_shapes(test)
    _, val_sh = synth.train_validation_split(train)
    is_val = [synth.shape_of_row(r) in set(val_sh) for r in tr_rows]
    tr_shapes = [problems[r] for r in tr_rows]
    t32 = T32.min(axis=1).astype(np.float64)
    n = pool.numel()
    for name, dt, eb, peak in (("bf16", kt.BF16, 2, 2500.0), ("fp8", kt.FP8E4M3, 1, 5000.0)):
        path = tune.table_path(name)
        if not os.path.exists(path):
            continue
        TL, PL, CL, metaL = tune.load_table(path)
        if not (TL >= 0).all() or [tuple(int(v) for v in p) for p in PL] != problems or \
                [tuple(c) for c in CL.tolist()] != h.kernels(dt)[:len(CL)] or \
                bool(metaL.get("pad_rows", False)) != pad:
            continue
        tl = TL.min(axis=1).astype(np.float64)
        ws_bytes = kt.Handle.prune_workspace_bytes(len(tr_rows), TL.shape[1], k, 10)
        pws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        sel = tune.select_pruning(h, TL[tr_rows], k, synth.SEED, workspace=pws, ws_bytes=ws_bytes,
                                  stream=stream)
        chosen = sel["chosen"]
        per_kind = {}
        h.set_fallback(0, dtype=dt)
        for kind in (0, 1, 2, 3):
            h.fit_selector(kind, tr_shapes, TL[tr_rows], chosen, mlp_steps=3000, mlp_graph_steps=25,
                           workspace=mws, ws_bytes=mws_bytes, stream=stream, dtype=dt)
            e = h.evaluate(TL, rows=te_rows, picks=[h.select(*problems[r], dtype=dt) for r in te_rows])
            per_kind[SEL_NAMES[kind]] = round(100 * e["geomean"], 2)
        h.set_fallback(1, dtype=dt)
        kind, vscores = h.fit_selector_validated(tr_shapes, TL[tr_rows], chosen, is_val,
                                                 mlp_steps=3000, mlp_graph_steps=25, workspace=mws,
                                                 ws_bytes=mws_bytes, stream=stream, dtype=dt)
        picks = [h.select(*p, dtype=dt) for p in problems]
        dep = h.evaluate(TL, rows=te_rows, picks=[picks[r] for r in te_rows])
        ceil = h.evaluate(TL, rows=te_rows, chosen=chosen)
        # operands in the low-precision format, converted on the GPU from the FP32 pool
        lp = torch.empty(n * eb + 256, dtype=torch.uint8, device="cuda")
        scales = torch.empty(4, dtype=torch.float32, device="cuda")
        if dt == kt.BF16:
            h.convert_bf16(pool, n, lp, stream=stream)
        else:
            h.quantize_fp8(pool, n, lp, scales, scales[2:], 8, stream=stream)
        base32, baselp = pool.data_ptr(), lp.data_ptr()

        def step(events=None):
            for i, pl in enumerate(plans):
                if events is not None:
                    events[i][0].record(stream)
                h.gemm_raw(dt, pl[0], 1.0, baselp + (pl[1] - base32) // 4 * eb, pl[2], pl[3],
                           baselp + (pl[4] - base32) // 4 * eb, pl[5], pl[6], 0.0, pl[7], pl[8],
                           pl[9], scaleA=scales.data_ptr(), scaleB=scales.data_ptr(),
                           config_id=-1, stream=stream)
                if events is not None:
                    events[i][1].record(stream)
        step()
        torch.cuda.synchronize()
        evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in plans] for _ in range(steps)]
        t0 = time.perf_counter()
        for s_ in range(steps):
            step(evs[s_])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        t_launch = np.array([[evs[s_][i][0].elapsed_time(evs[s_][i][1]) for i in range(len(plans))]
                             for s_ in range(steps)]).mean(axis=0)
        inst = {}
        for i, p in enumerate(problems):
            if h.get_kernel(picks[i], dt)[0][4] > 1:     # split-K picks run several kernels
                continue
            key = (picks[i], p[4], p[5])
            inst[key] = inst.get(key, 0.0) + t_launch[i]
        dom = max(inst, key=inst.get)
        dom_rows = [i for i, p in enumerate(problems) if (picks[i], p[4], p[5]) == dom]
        dom_tf = float(flops[dom_rows].sum()) / (float(t_launch[dom_rows].sum()) * 1e-3) / 1e12
        bm, bn, tt, bk = h.get_kernel(dom[0], dt)[0][:4]
        out[name] = {
            "live_tflops": round(float(flops.sum()) / (ms * 1e-3) / 1e12, 2),
            "ms_per_step": round(ms, 3),
            "exhaustive_best_tflops": round(float(flops.sum()) / (tl.sum() * 1e-9) / 1e12, 2),
            "speedup_vs_f32_best_geomean": round(_geomean(t32 / tl), 3),
            "speedup_vs_f32_best_time_weighted": round(float(t32.sum() / tl.sum()), 3),
            "deployed_selector": SEL_NAMES[kind],
            "deployed_pct_of_optimal_test": round(100 * dep["geomean"], 2),
            "deployed_frac_ge_0.9_test": round(dep["frac_ge_0_9"], 4),
            "selector_pct_of_optimal_test": per_kind,
            "selector_validation_scores": {SEL_NAMES[i]: round(100 * v, 2) for i, v in enumerate(vscores)},
            "kmeans_ceiling_test": round(100 * ceil["geomean"], 2),
            "chosen": [list(h.get_kernel(c, dt)[0]) for c in chosen],
            "normalization": sel["norm_name"], "train_ceiling_by_normalization": sel["train_ceiling"],
            "accuracy_bound_rel_frobenius": 1e-2 if dt == kt.BF16 else 4e-2,
            "roofline": {"bound": "mfma", "kernel": f"gemm_lp{'_dma' if pad else ''}_kernel<{eb}, "
                                                    f"{bm}, {bn}, {tt}, {bk}, "
                                                    f"{dom[1]}, {dom[2]}>",
                         "launches_per_step": len(dom_rows), "achieved": round(dom_tf, 2),
                         "peak": peak, "unit": "TFLOP/s", "frac": round(dom_tf / peak, 4),
                         "kernel_ms_per_step": round(float(t_launch[dom_rows].sum()), 3)},
        }
        del lp
    return out


def square_lp_section(kt, h, torch, synth, stream, n=4096, reps=10):
    """BF16 and FP8 on one large square product (n^3, batch 1, alpha 1,
    beta 0) in the four layouts: the fastest of the configurations with
    tiles of at least 128 x 128 (an exhaustive search over that subset),
    operands with 16-byte rows (the LDS-DMA pipeline), HIP events over `reps`
    launches on the launch stream; fraction of the dtype's dense MFMA peak."""
    out = {}
    M = N = K = n
    src = torch.empty(n * n, dtype=torch.float32, device="cuda")
    h.fill_uniform(src, src.numel(), synth.operand_seed(synth.SEED + 5, 0), stream=stream)
    C = torch.empty(n * n, dtype=torch.float32, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name, dt, eb, peak in (("bf16", kt.BF16, 2, 2500.0), ("fp8", kt.FP8E4M3, 1, 5000.0)):
        A = torch.empty(n * n * eb, dtype=torch.uint8, device="cuda")
        B = torch.empty(n * n * eb, dtype=torch.uint8, device="cuda")
        sc = torch.ones(4, dtype=torch.float32, device="cuda")
        if dt == kt.BF16:
            h.convert_bf16(src, n * n, A, stream=stream)
            h.convert_bf16(src, n * n, B, stream=stream)
        else:
            amax = torch.zeros(4, dtype=torch.int32, device="cuda")
            h.quantize_fp8(src, n * n, A, sc[0:], amax, 16, stream=stream)
            h.quantize_fp8(src, n * n, B, sc[1:], amax, 16, stream=stream)
        cfgs = h.configs(dt)
        cand = [i for i, c in enumerate(cfgs) if c[0] * c[1] >= 128 * 128]
        res = {}
        for ta, tb in synth.LAYOUTS:
            lda, ldb = (M if ta else K), (K if tb else N)
            shp = kt.shape(M, N, K, 1, ta, tb)
            assert h.dma_pipeline(dt, shp, A, lda, 0, B, ldb, 0)

            def run(cid):
                h.gemm_raw(dt, shp, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, N, 0,
                           scaleA=sc[0:].data_ptr(), scaleB=sc[1:].data_ptr(), config_id=cid,
                           stream=stream)
            best = None
            for cid in cand:
                run(cid)
                e0.record(stream)
                for _ in range(3):
                    run(cid)
                e1.record(stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / 3
                if best is None or ms < best[0]:
                    best = (ms, cid)
            cid = best[1]
            run(cid)
            e0.record(stream)
            for _ in range(reps):
                run(cid)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = 2.0 * M * N * K / (ms * 1e-3) / 1e12
            res["%d%d" % (ta, tb)] = {"config": list(cfgs[cid]), "us": round(ms * 1e3, 1),
                                      "tflops": round(tf, 1), "frac_of_peak": round(tf / peak, 4)}
        out[name] = res
        del A, B
    return {"n": n, "layouts_transA_transB": out}


def conv_section(kt, h, tune, problems_conv_path, sel_kinds, fit_args):
    """Held-out generalization: the GEMMs of a VGG16-style conv stack (im2col
    and Winograd lowerings, never seen in training) through the selectors
    fitted on the sweep set, measured against their own exhaustive sweep."""
    if not os.path.exists(problems_conv_path):
        return None
    TC, PC, CC, metaC = tune.load_table(problems_conv_path)
    if not (TC >= 0).all() or TC.shape[1] != fit_args[1].shape[1]:
        return None   # incomplete, or measured over other kernels than the sweep table
    probs = [tuple(int(v) for v in p) for p in PC]
    F = np.array([2.0 * p[0] * p[1] * p[2] * p[3] for p in probs])
    tb = TC.min(axis=1).astype(np.float64)
    out = {"problems": len(probs), "gflop": round(float(F.sum()) / 1e9, 1),
           "exhaustive_best_tflops": round(float(F.sum()) / (tb.sum() * 1e-9) / 1e12, 2)}
    tr_shapes, T_tr, chosen, mws, mws_bytes, stream = fit_args
    for kind in sel_kinds:
        h.fit_selector(kind, tr_shapes, T_tr, chosen, mlp_steps=3000, mlp_graph_steps=25,
                       workspace=mws, ws_bytes=mws_bytes, stream=stream)
        picks = [h.select(*p) for p in probs]
        ts = TC[np.arange(len(probs)), picks].astype(np.float64)
        out[SEL_NAMES[kind]] = {"pct_of_optimal_geomean": round(100 * _geomean(tb / ts), 2),
                                "selected_tflops_table": round(float(F.sum()) / (ts.sum() * 1e-9) / 1e12, 2)}
    ceil = np.array([TC[i, chosen].min() for i in range(len(probs))], dtype=np.float64)
    out["kmeans_ceiling_pct"] = round(100 * _geomean(tb / ceil), 2)
    return out


def calibrate_counters(log2n=28, reps=3):
    """A kernel of known HBM traffic for scaling rocprofv3's FETCH_SIZE and
    WRITE_SIZE: the library's BF16 conversion reads 4 bytes and writes 2
    bytes per element, each once, on a buffer far larger than the caches.
    Run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) and divide the
    printed bytes per dispatch by the counter's reading."""
    import torch

    import paper_2008_13145_amd as kt
    n = 1 << log2n
    h = kt.Handle(0)
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    h.fill_uniform(x, n, 1)
    y = torch.empty(n, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    for _ in range(reps):
        h.convert_bf16(x, n, y)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"kernel": "cvt_bf16_kernel", "elements": n, "fetch_bytes": 4 * n,
                      "write_bytes": 2 * n, "dispatches": reps}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--selector", default="auto", choices=["auto", "DT-A", "DT-B", "DT-C", "MLP"],
                    help="auto: the kind that scores best on validation shapes of the training set")
    ap.add_argument("--table", default=None)
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowp", action="store_true", help="skip the BF16/FP8 sections")
    ap.add_argument("--calibrate-counters", action="store_true",
                    help="only run the known-traffic conversion kernel (HBM counter scaling)")
    ap.add_argument("--step-only", action="store_true",
                    help="only pruning, the deployed selector and the timed steps (for counter "
                         "runs: the dominant kernel's last dispatches are the timed step's)")
    ap.add_argument("--grouped-only", action="store_true",
                    help="only the grouped BF16 section (for profiling its kernel)")
    ap.add_argument("--square-only", action="store_true",
                    help="only the BF16 / FP8 4096^3 section (for profiling its kernels)")
    a = ap.parse_args(argv)
    if a.calibrate_counters:
        calibrate_counters()
        return 0
    if a.grouped_only:
        import torch

        import paper_2008_13145_amd as kt
        import synth
        h = kt.Handle(0)
        print(json.dumps(grouped_section(kt, h, torch, synth, torch.cuda.current_stream())),
              flush=True)
        h.close()
        return 0
    if a.square_only:
        import torch

        import paper_2008_13145_amd as kt
        import synth
        h = kt.Handle(0)
        print(json.dumps(square_lp_section(kt, h, torch, synth, torch.cuda.current_stream())),
              flush=True)
        h.close()
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); sharding the "
              "path over several GPUs is not built", file=sys.stderr)
        return 2

    import torch

    import paper_2008_13145_amd as kt
    import synth
    from paper_2008_13145_amd import tune

    table_path = a.table or tune.DEFAULT_TABLE
    if not os.path.exists(table_path):
        raise SystemExit(f"benchmark table {table_path} missing: run "
                         "`python -m paper_2008_13145_amd.tune sweep` on the GPU first")
    T, P, C, meta = tune.load_table(table_path)
    problems = [tuple(int(v) for v in p) for p in P]
    if not (T >= 0).all():
        raise SystemExit("benchmark table is incomplete; resume the sweep")
    n_prob, n_cfg = T.shape
    train, test = synth.train_test_split()
    tr_rows = synth.rows_of_shapes(train)
    te_rows = synth.rows_of_shapes(test)

    h = kt.Handle(0)
    kernels = h.kernels()
    assert [tuple(c) for c in C.tolist()] == kernels[:n_cfg], "table columns are not this build's kernels"
    # the operand layout the table was measured with: rows padded to 16
    # elements (allocated in full, promised to the library) or dense; the
    # fallback's timings below use it too
    pad = bool(meta.get("pad_rows", False))
    h.set_full_rows(pad)
    # partial planes for the split-K kernels kt_gemm runs (selected or forced)
    gemm_ws = torch.empty(kt.SPLIT_PLANE_CAP, dtype=torch.uint8, device="cuda")
    h.set_workspace(gemm_ws)
    _log(f"bench: table {table_path} ({n_prob} problems x {n_cfg} configs)")
    stream = torch.cuda.current_stream()

    # ---- pruning (GPU k-means on the training rows) and the Top-N baseline
    k = a.k
    ws_bytes = kt.Handle.prune_workspace_bytes(len(tr_rows), n_cfg, max(k, 15), 10)
    pws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    # the normalization (section 3.4) is chosen on the training rows
    sel = tune.select_pruning(h, T[tr_rows], k, synth.SEED, workspace=pws, ws_bytes=ws_bytes,
                              stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = h.prune(T[tr_rows], k, norm=sel["norm"], seed=synth.SEED, n_init=10, max_iter=300,
                 workspace=pws, ws_bytes=ws_bytes, stream=stream)
    prune_ms = (time.perf_counter() - t0) * 1e3
    chosen = pr["chosen"]
    assert chosen == sel["chosen"]
    _log(f"bench: pruned to {chosen} ({sel['norm_name']} normalization) in {prune_ms:.1f} ms")
    topn = h.prune_topn(T[tr_rows], k, workspace=pws, ws_bytes=ws_bytes, stream=stream)

    def ev_ceiling(ch, rows=te_rows):      # section 4.3 through kt_evaluate
        return h.evaluate(T, rows=rows, chosen=ch)

    def ev_picks(picks, rows=te_rows):
        return h.evaluate(T, rows=rows, picks=picks)

    evals, frac09, summaries = {}, {}, {}

    def record(name, e):
        evals[name] = e["geomean"]
        frac09[name] = round(e["frac_ge_0_9"], 4)
        summaries[name] = {"mean": round(100 * e["mean"], 2), "min": round(100 * e["min"], 2)}

    record("kmeans_ceiling", ev_ceiling(chosen))
    record("topn_ceiling", ev_ceiling(topn))
    # single best kernel over the training rows (no selector at all)
    single = max(range(n_cfg), key=lambda c: ev_picks([c] * len(tr_rows), tr_rows)["geomean"])
    record("single_kernel", ev_picks([single] * len(te_rows)))

    # ---- selectors fitted on the training rows, each scored by its own
    # pick on the held-out rows (the out-of-range fallback off)
    tr_shapes = [problems[r] for r in tr_rows]
    fit_ms = {}
    # sized for the largest k of the comparison over k below
    mws_bytes = kt.Handle.mlp_workspace_bytes(len(tr_rows), n_cfg, max(k, 15))
    mws = torch.empty(mws_bytes, dtype=torch.uint8, device="cuda")
    h.set_fallback(0)
    for kind in (() if a.step_only else (0, 1, 2, 3)):
        t0 = time.perf_counter()
        h.fit_selector(kind, tr_shapes, T[tr_rows], chosen, mlp_steps=3000, mlp_graph_steps=25,
                       workspace=mws, ws_bytes=mws_bytes, stream=stream)
        torch.cuda.synchronize()
        fit_ms[SEL_NAMES[kind]] = (time.perf_counter() - t0) * 1e3
        record(SEL_NAMES[kind], ev_picks([h.select(*problems[r]) for r in te_rows]))
    infer_mlp = None if a.step_only else \
        selection_latency(kt, h, torch, problems, stream)    # h holds the MLP here
    h.set_fallback(1)
    conv = None if a.step_only else \
        conv_section(kt, h, tune, tune.table_path("f32", "conv"), (0, 1, 2, 3),
                     (tr_shapes, T[tr_rows], chosen, mws, mws_bytes, stream))

    # ---- the paper's comparison over the number of deployed kernels: for
    # each k, pruning (normalization chosen on the training rows), Top-N and
    # decision tree B, scored on the held-out rows (a separate handle, so the
    # deployed selector above is untouched)
    k_sweep = {}
    hk = kt.Handle(0)
    hk.set_fallback(0)
    for kk in (() if a.step_only else (4, 5, 6, 8, 15)):
        s_k = tune.select_pruning(hk, T[tr_rows], kk, synth.SEED, workspace=pws,
                                  ws_bytes=ws_bytes, stream=stream)
        tn_k = hk.prune_topn(T[tr_rows], kk, workspace=pws, ws_bytes=ws_bytes, stream=stream)
        hk.fit_selector(kt.SEL_DT_B, tr_shapes, T[tr_rows], s_k["chosen"])
        picks_k = [hk.select(*problems[r]) for r in te_rows]
        hk.fit_selector(kt.SEL_MLP, tr_shapes, T[tr_rows], s_k["chosen"], mlp_steps=3000,
                        mlp_graph_steps=25, workspace=mws, ws_bytes=mws_bytes, stream=stream)
        picks_m = [hk.select(*problems[r]) for r in te_rows]
        k_sweep[str(kk)] = {
            "normalization": s_k["norm_name"],
            "kmeans_ceiling": round(100 * ev_ceiling(s_k["chosen"])["geomean"], 2),
            "topn_ceiling": round(100 * ev_ceiling(tn_k)["geomean"], 2),
            "DT-B": round(100 * ev_picks(picks_k)["geomean"], 2),
            "MLP": round(100 * ev_picks(picks_m)["geomean"], 2)}
    # ---- sparse-sampled tuning: prune from a random fraction of the
    # training table's entries (the rest unmeasured), score on the held-out
    # rows of the full table
    sparse = {}
    rng_s = np.random.default_rng(synth.SEED + 7)
    for frac in (() if a.step_only else (0.05, 0.1, 0.25, 0.5, 1.0)):
        T_s = T[tr_rows].copy()
        T_s[rng_s.random(T_s.shape) >= frac] = -1
        ch_s = hk.prune(T_s, k, norm=sel["norm"], seed=synth.SEED, n_init=10, max_iter=300,
                        workspace=pws, ws_bytes=ws_bytes, stream=stream)["chosen"]
        sparse[str(frac)] = round(100 * ev_ceiling(ch_s)["geomean"], 2)
    # ---- pruning in a reduced space: principal components of the normalized
    # training table, then the same k-means; each centroid read back through
    # the components (the paper's representative rule)
    pca = {}
    for dims in (() if a.step_only else (8, 16, 32)):
        r_p = tune.pca_pruning(hk, T[tr_rows], k, synth.SEED, dims, sel["norm"], workspace=pws,
                               ws_bytes=ws_bytes, stream=stream)
        pca[str(dims)] = {"explained_variance": round(r_p["explained"], 4),
                          "kmeans_ceiling": round(100 * ev_ceiling(r_p["chosen"])["geomean"], 2)}
    # ---- the pruner grid (section 4.3's comparison): every pruning method
    # under every normalization, with both of section 4.2's cluster -> kernel
    # rules (representative / geometric mean of the members), ceiling on the
    # held-out rows
    def ceil_test(ch):
        return round(100 * ev_ceiling(ch)["geomean"], 2)
    grid = {"top_n": ceil_test(topn)}
    for norm, name in enumerate(() if a.step_only else tune.NORM_NAMES):
        cell = {}
        for rep, rname in ((0, "centroid"), (1, "geomean_of_members")):
            cell[f"kmeans_{rname}"] = ceil_test(tune.kmeans_pruning(
                hk, T[tr_rows], k, synth.SEED, norm, rep=rep, workspace=pws, ws_bytes=ws_bytes,
                stream=stream))
            cell[f"pca16_kmeans_{rname}"] = ceil_test(tune.pca_pruning(
                hk, T[tr_rows], k, synth.SEED, 16, norm, rep=2 if rep == 0 else 1, workspace=pws,
                ws_bytes=ws_bytes, stream=stream)["chosen"])
            cell[f"decision_tree_{'leaf_mean' if rep == 0 else rname}"] = ceil_test(
                tune.tree_pruning(hk, T[tr_rows], tr_shapes, k, norm, rep=rep, stream=stream))
        grid[name] = cell
    hk.close()
    _log(f"bench: k sweep {json.dumps(k_sweep)}; sparse sampling {json.dumps(sparse)}; "
         f"pca {json.dumps(pca)}; pruner grid {json.dumps(grid)}")

    # ---- the deployed selector: chosen among trees A/B/C and the MLP on
    # validation shapes carved out of the training shapes (never the test
    # shapes), refitted on all training rows; the out-of-range fallback on
    fit_sh, val_sh = synth.train_validation_split(train)
    val_set = set(val_sh)
    is_val = [synth.shape_of_row(r) in val_set for r in tr_rows]
    if a.selector == "auto":
        sel_kind, val_scores = h.fit_selector_validated(
            tr_shapes, T[tr_rows], chosen, is_val, mlp_steps=3000, mlp_graph_steps=25,
            workspace=mws, ws_bytes=mws_bytes, stream=stream)
    else:
        sel_kind = {v: kk for kk, v in SEL_NAMES.items()}[a.selector]
        h.fit_selector(sel_kind, tr_shapes, T[tr_rows], chosen, mlp_steps=3000,
                       mlp_graph_steps=25, workspace=mws, ws_bytes=mws_bytes, stream=stream)
        val_scores = None
    torch.cuda.synchronize()
    sel_name = SEL_NAMES[sel_kind]
    _log(f"bench: deployed selector {sel_name} (validation scores {val_scores})")
    picks_all = [h.select(*p) for p in problems]       # fallback timing happens here, once
    deployed_te = ev_picks([picks_all[r] for r in te_rows])
    # the split-K kernel family (section 3's kernel type for deep, under-
    # filled products): where it is the exhaustive best, where the deployed
    # selector runs it, and the held-out deep-K under-filled rows
    n_cfg_plain = h.num_configs()
    best_col = T.argmin(axis=1)

    def underfilled(r):
        M_, N_, K_, b_ = problems[r][:4]
        bm_, bn_ = kernels[int(best_col[r])][:2]
        return K_ >= 512 and -(-M_ // bm_) * -(-N_ // bn_) * b_ < 256
    uf_te = [r for r in te_rows if underfilled(r)]
    split_family = {
        "kernels": n_cfg - n_cfg_plain,
        "chosen_split_kernels": [list(kernels[c]) for c in chosen if c >= n_cfg_plain],
        "rows_split_best": int((best_col >= n_cfg_plain).sum()),
        "rows_split_best_by_5pct": int(sum(1 for r in range(n_prob) if best_col[r] >= n_cfg_plain and
                                           T[r, :n_cfg_plain].min() > 1.05 * T[r].min())),
        "test_rows_running_split": int(sum(1 for r in te_rows if picks_all[r] >= n_cfg_plain)),
        "underfilled_deep_k_test_rows": len(uf_te)}
    if uf_te:
        split_family["underfilled_deep_k_test_pct_of_optimal"] = round(
            100 * ev_picks([picks_all[r] for r in uf_te], uf_te)["geomean"], 2)
        split_family["underfilled_deep_k_test_ceiling_pct"] = round(
            100 * ev_ceiling(chosen, uf_te)["geomean"], 2)
        split_family["underfilled_deep_k_test_ceiling_chosen_minus_split_kernels_pct"] = round(
            100 * h.evaluate(T[:, :n_cfg_plain], rows=uf_te,
                             chosen=[c for c in chosen if c < n_cfg_plain] or [0])["geomean"], 2)
    box = h.selector_info()
    n_outside = sum(1 for r in te_rows if any(
        not (box["box_lo"][f] <= problems[r][f] <= box["box_hi"][f]) for f in range(4)))
    t0 = time.perf_counter()
    for _ in range(5):
        for p in problems:
            h.select(*p)
    select_us = (time.perf_counter() - t0) / (5 * n_prob) * 1e6
    sel_all = ev_picks(picks_all, list(range(n_prob)))
    infer = None if a.step_only else \
        {"deployed": selection_latency(kt, h, torch, problems, stream), "MLP": infer_mlp}

    # ---- operands resident in HBM: one pool sized for the largest problem
    ws_all = kt.Handle.sweep_workspace_bytes(problems)
    pool = torch.empty(ws_all // 4 + 64, dtype=torch.float32, device="cuda")
    h.fill_uniform(pool, pool.numel(), synth.operand_seed(synth.SEED, 0), stream=stream)
    base = pool.data_ptr()
    rnd = (lambda v: (v + 15) // 16 * 16) if pad else (lambda v: v)
    plans = []
    for (M, N, K, b, ta, tb) in problems:
        lda = rnd(M if ta else K)
        ldb = rnd(K if tb else N)
        sA, sB, sC = (K if ta else M) * lda, (N if tb else K) * ldb, M * N
        offB = ((b * sA * 4 + 255) // 256) * 256
        offC = offB + ((b * sB * 4 + 255) // 256) * 256
        plans.append((kt.shape(M, N, K, b, ta, tb), base, lda, sA, base + offB, ldb, sB,
                      base + offC, N, sC))
    flops = np.array([2.0 * p[0] * p[1] * p[2] * p[3] for p in problems])
    total_flops = float(flops.sum())

    def step(events=None):
        for i, pl in enumerate(plans):
            if events is not None:
                events[i][0].record(stream)
            h.gemm_raw(kt.F32, pl[0], 1.0, pl[1], pl[2], pl[3], pl[4], pl[5], pl[6], 0.0, pl[7],
                       pl[8], pl[9], config_id=-1, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    _log("bench: selectors fitted; warm-up")
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in problems] for _ in range(a.steps)]
    torch.cuda.synchronize()
    # (not in --step-only runs, which run under the profiler: rocm-smi is a
    # child process and the profiler's preload would follow it)
    state_before = None if a.step_only else gpu_state()
    t_start = time.perf_counter()
    for s in range(a.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    state_after = None if a.step_only else gpu_state()
    ms_per_step = wall * 1e3 / a.steps
    per_launch = np.array([[evs[s][i][0].elapsed_time(evs[s][i][1]) for i in range(n_prob)]
                           for s in range(a.steps)])          # ms
    t_launch = per_launch.mean(axis=0)
    value = total_flops / (ms_per_step * 1e-3) / 1e12

    # dominant kernel: the (configuration, layout) instantiation with the most time
    cfgs = kernels
    inst_time = {}
    for i, p in enumerate(problems):
        if cfgs[picks_all[i]][4] > 1:     # split-K picks run several kernels
            continue
        key = (picks_all[i], p[4], p[5])
        inst_time[key] = inst_time.get(key, 0.0) + t_launch[i]
    dom = max(inst_time, key=inst_time.get)
    dom_rows = [i for i, p in enumerate(problems) if (picks_all[i], p[4], p[5]) == dom]
    dom_flops = float(flops[dom_rows].sum())
    dom_bytes = float(sum(4.0 * problems[i][3] * (problems[i][0] * problems[i][2] +
                                                  problems[i][2] * problems[i][1] +
                                                  problems[i][0] * problems[i][1]) for i in dom_rows))
    dom_ms = float(t_launch[dom_rows].sum())
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    bm, bn, tt, bk = cfgs[dom[0]][:4]
    # padded rows put every operand on the LDS-DMA pipeline where the
    # configuration has one (t >= 2, tiles of whole KiB)
    dma = pad and tt >= 2 and (bm * bk * 4) % 1024 == 0 and (bn * bk * 4) % 1024 == 0
    dom_name = f"gemm_f32{'_dma' if dma else ''}_kernel<{bm}, {bn}, {tt}, {bk}, {dom[1]}, {dom[2]}>"

    # exhaustive-best comparison: live launch times vs the table's best
    t_best = T.min(axis=1).astype(np.float64)
    pct_exh_live = float(t_best.sum() * 1e-6 / t_launch.sum())
    out = {
        "metric": "GEMM TFLOP/s; % of exhaustive-best config; % MFMA peak; selector regret",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sweep set: 300 seeded log-uniform (M,N,K in 16..4096, batch 1..64) x 4 "
                        "layouts = 1200 FP32 GEMMs, alpha 1, beta 0; each run through the "
                        f"deployed path (selector {sel_name} over k={k} k-means-pruned kernels)",
            "problems": n_prob, "gflop_per_step": round(total_flops / 1e9, 3),
            "k": k, "selector": sel_name, "selector_choice": a.selector,
            "selector_validation_scores": None if val_scores is None else
            {SEL_NAMES[i]: round(100 * v, 2) for i, v in enumerate(val_scores)},
            "chosen": [list(cfgs[c]) for c in chosen],
            "normalization": sel["norm_name"], "train_ceiling_by_normalization": sel["train_ceiling"],
            "train_test_shapes": [len(train), len(test)],
        },
        "pct_mfma_peak": round(100 * value / FP32_PEAK_TFLOPS, 2),
        # the target figure: geometric mean over the held-out shapes of
        # t_best / t_selected, deployed selector with its fallback
        "deployed_pct_of_optimal_test": {
            "geomean": round(100 * deployed_te["geomean"], 2),
            "mean": round(100 * deployed_te["mean"], 2), "min": round(100 * deployed_te["min"], 2),
            "frac_ge_0.9": round(deployed_te["frac_ge_0_9"], 4),
            "test_rows_outside_training_range": n_outside, "target_met": deployed_te["geomean"] >= 0.9},
        "split_k_family": split_family,
        "pct_of_exhaustive_best": {
            "geomean_all_rows_table_in_sample": round(100 * sel_all["geomean"], 2),
            "time_weighted_live_in_sample": round(100 * pct_exh_live, 2),
        },
        "selector_pct_of_optimal_test": {kk: round(100 * v, 2) for kk, v in evals.items()},
        "selector_mean_min_pct_test": summaries,
        "selector_regret_test": {kk: round(1 - v, 4) for kk, v in evals.items()},
        "selector_frac_ge_0.9_test": frac09,
        "select_us_per_call": round(select_us, 3),
        "selection_latency": infer,
        "prune_ms_gpu": round(prune_ms, 2),
        "fit_ms": {kk: round(v, 1) for kk, v in fit_ms.items()},
        "roofline": {
            "bound": "mfma", "kernel": dom_name, "launches_per_step": len(dom_rows),
            "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(dom_name),
            "algorithmic_bytes_per_launch": int(dom_bytes / len(dom_rows)),
            "kernel_ms_per_step": round(dom_ms, 3),
        },
        "operand_rows": "padded to 16 elements" if pad else "dense",
        "table": {"path": os.path.relpath(table_path, ROOT), "device": meta.get("device"),
                  "sweep_seconds": round(meta.get("seconds", 0.0), 1)},
        "deploy": deploy_info(chosen, [h.num_configs(d) for d in (kt.F32, kt.BF16, kt.FP8E4M3)]),
        "k_sweep_pct_of_optimal_test": k_sweep,
        "sparse_sampling_kmeans_ceiling_test": sparse,
        "pca_kmeans_ceiling_test": pca,
        "pruner_grid_ceiling_test": grid,
        "gpu_state": {"before": state_before, "after": state_after},
    }
    _log(f"bench: {value:.2f} TFLOP/s, {ms_per_step:.1f} ms/step")
    if a.step_only:
        # the dominant configuration's problems in each layout, in launch order
        out["dominant_config_problems"] = {
            f"{ta}{tb}": [list(problems[i]) for i in range(n_prob)
                          if picks_all[i] == dom[0] and problems[i][4:6] == (ta, tb)]
            for ta in (0, 1) for tb in (0, 1)}
        h.close()
        print(json.dumps(out), flush=True)
        return 0
    if conv:
        out["conv_heldout"] = conv
    if not a.no_lowp:
        lp = lowp_section(kt, h, torch, tune, synth, problems, T, pool, plans, flops, k, 3, stream,
                          mws, mws_bytes, pad=pad)
        if lp:
            out["lowp"] = lp
            _log(f"bench: low precision {json.dumps(lp)}")
    out["single_gemm_256"] = single_gemm_section(kt, h, torch, synth, stream)
    out["repeatability"] = repeatability(kt, h, torch, T, problems, plans, stream)
    out["split_k"] = splitk_section(kt, h, torch, T, problems, plans, chosen, stream)
    _log(f"bench: split-K {json.dumps(out['split_k'])}")
    out["vgg16"] = vgg16_section(kt, h, torch, synth, stream)
    _log(f"bench: VGG16 {json.dumps(out['vgg16']['ms_per_inference'])}, "
         f"{out['vgg16']['selector_pct_of_exhaustive']} % of exhaustive")
    _log(f"bench: single GEMM {json.dumps(out['single_gemm_256'])}; repeatability "
         f"{json.dumps(out['repeatability'])}")
    if not a.no_lowp:
        out["square_lp_4096"] = square_lp_section(kt, h, torch, synth, stream)
        _log(f"bench: 4096^3 {json.dumps(out['square_lp_4096'])}")
        out["grouped_bf16"] = grouped_section(kt, h, torch, synth, stream)
        _log(f"bench: grouped {json.dumps(out['grouped_bf16'])}")
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problems, a.cpu_budget_s,
                                           tuning=(T[tr_rows], tr_shapes, sel["norm"], k))
    h.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
