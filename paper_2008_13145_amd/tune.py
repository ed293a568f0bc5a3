"""Offline tuning driver: the benchmark sweep that builds the dataset the
pruning and selection learn from (sections 3 and 3.1 of the paper), and the
deploy build that keeps only the pruned kernels (section 4).

    python -m paper_2008_13145_amd.tune sweep --out TABLE.npz [--budget-s 900]
    python -m paper_2008_13145_amd.tune deploy --table TABLE.npz --k 8

The sweep is resumable: the table is saved after every chunk of rows, and a
restart skips rows already measured (entries >= 0).  Problems are the 300
seeded log-uniform shapes of ``synth.sweep_shapes()`` in all four layouts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "data", "sweep_f32_mi355x.npz")
DTYPE_NAMES = {"f32": 0, "bf16": 1, "fp8": 2}


def table_path(dtype_name: str, problem_set: str = "sweep") -> str:
    return os.path.join(HERE, "data", f"{problem_set}_{dtype_name}_mi355x.npz")


def problem_set(name: str):
    """Problems of a named set: 'sweep' (300 shapes x 4 layouts) or 'conv' (the
    GEMMs of a VGG16-style conv stack, im2col and Winograd lowerings, NN)."""
    import synth
    if name == "sweep":
        return synth.sweep_problems()
    if name == "conv":
        return [(c["M"], c["N"], c["K"], c["batch"], 0, 0) for c in synth.conv_shapes()]
    raise ValueError(name)
DEPLOY_SPEC = os.path.join(HERE, "data", "deploy_f32.json")
DEPLOY_LIB = os.path.join(HERE, "libkt_deploy.so")


NORM_NAMES = ("relative", "raw_cutoff", "std_cutoff", "sigmoid")
REP_NAMES = {0: "mean", 1: "geomean", 2: "centroid"}


def select_pruning(h, T_train, k, seed, n_init=10, max_iter=300, workspace=None, ws_bytes=0,
                   stream=None):
    """k-means pruning (section 4.1) under the normalization of section 3.4
    whose chosen set keeps the most of the optimum on the training rows
    (kt_prune_auto).  Returns {"norm", "norm_name", "chosen",
    "train_ceiling": {name: score}}."""
    r = h.prune_auto(T_train, k, seed=seed, n_init=n_init, max_iter=max_iter,
                     workspace=workspace, ws_bytes=ws_bytes, stream=stream)
    return {"norm": r["norm"], "norm_name": NORM_NAMES[r["norm"]], "chosen": r["chosen"],
            "train_ceiling": {name: round(v, 6) for name, v in zip(NORM_NAMES, r["scores"])}}


def normalized_table(h, T, norm, stream=None):
    """The Q16 normalized table (section 3.4) computed on the GPU, as a host
    uint16 array."""
    import torch
    T = np.ascontiguousarray(T, dtype=np.int64)
    n, d = T.shape
    dT = torch.from_numpy(T).cuda()
    out = torch.zeros((n, d), dtype=torch.int16, device="cuda")
    h.normalize(dT, n, d, norm, out, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint16)


def tree_pruning(h, T_train, shapes, k, norm, rep=0, stream=None):
    """Decision-tree pruning (section 4.1) on the GPU-normalized table: the
    leaves' rounded means pick the kernels (rep 0, kt_prune_tree) or their
    members' geometric means (rep 1, section 4.2's rule for label-only
    clusters)."""
    Xq = normalized_table(h, T_train, norm, stream)
    if rep == 0:
        return h.prune_tree(shapes, Xq, k)
    labels, n_leaves = h.prune_tree_leaves(shapes, Xq, k)
    return h.representatives(Xq, labels, n_leaves, k, rep)


def kmeans_pruning(h, T_train, k, seed, norm, rep=0, n_init=10, max_iter=300, workspace=None,
                   ws_bytes=0, stream=None):
    """k-means pruning (section 4.1): each centroid's best configuration
    (rep 0, kt_prune) or the best for its members' geometric mean (rep 1)."""
    r = h.prune(T_train, k, norm=norm, seed=seed, n_init=n_init, max_iter=max_iter,
                workspace=workspace, ws_bytes=ws_bytes, stream=stream)
    if rep == 0:
        return r["chosen"]
    return h.representatives(normalized_table(h, T_train, norm, stream), r["labels"], k, k, rep)


def pca_pruning(h, T_train, k, seed, dims, norm, rep=2, n_init=10, max_iter=300, workspace=None,
                ws_bytes=0, stream=None):
    """PCA + k-means pruning (section 4.1, kt_prune_pca): the leading `dims`
    principal components of the normalized training rows, the library's
    integer k-means on their 16-bit quantization, and each cluster's kernel
    from its centroid read back in the original coordinates (rep 2) or from
    its members' geometric mean (rep 1).  Returns {"chosen", "inertia",
    "explained", "labels"}."""
    return h.prune_pca(T_train, k, norm, dims, rep=rep, seed=seed, n_init=n_init,
                       max_iter=max_iter, workspace=workspace, ws_bytes=ws_bytes, stream=stream)


def load_table(path):
    """(time_ns int64 [P][C], problems int64 [P][6], kernels int32 [C][5], meta
    dict).  Column c is kernel id c; a kernel row is (bm, bn, t, bk, slices)
    (tables that hold configurations only have slices 1 added)."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        C = z["configs"].copy()
        if C.shape[1] == 4:
            C = np.concatenate([C, np.ones((C.shape[0], 1), C.dtype)], axis=1)
        return z["time_ns"].copy(), z["problems"].copy(), C, meta


def save_table(path, time_ns, problems, configs, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, time_ns=time_ns, problems=np.asarray(problems, np.int64),
                        configs=np.asarray(configs, np.int32), meta=np.array(json.dumps(meta)))
    os.replace(tmp, path)


def run_sweep(out, budget_s=900.0, target_ms=5.0, min_reps=3, max_reps=200,
              cut_factor=8.0, warmup=2, limit=None, log=print, dtype=0, set_name="sweep",
              pad_rows=True):
    import torch

    import synth
    from . import Handle
    h = Handle(0)
    problems = problem_set(set_name)
    if limit:
        problems = problems[:limit]
    configs = h.kernels(dtype)     # every kernel: configurations, then split-K variants
    if os.path.exists(out):
        T, P, C, meta = load_table(out)
        if P.tolist() != [list(p) for p in problems] or C.tolist() != [list(c) for c in configs]:
            raise RuntimeError(f"{out} was made for another problem set or configuration space")
        if bool(meta.get("pad_rows", False)) != pad_rows:
            raise RuntimeError(f"{out} was measured with another operand layout")
    else:
        T = np.full((len(problems), len(configs)), -1, np.int64)
        props = torch.cuda.get_device_properties(0)
        meta = dict(device=props.name, arch=getattr(props, "gcnArchName", ""),
                    opts=dict(target_ms=target_ms, min_reps=min_reps, max_reps=max_reps,
                              cut_factor=cut_factor, warmup=warmup),
                    seed=synth.SEED, started=time.time(), seconds=0.0, dtype=dtype,
                    pad_rows=bool(pad_rows))
    ws_bytes = Handle.sweep_workspace_bytes(problems, dtype)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    # Load every kernel once on a tiny problem, so that no row pays for code
    # object loading and the first timed launch of a pair is representative.
    tiny = [(16, 16, 16, 1, ta, tb) for (ta, tb) in synth.LAYOUTS]
    for pad in (False, True):     # both pipelines of every kernel
        h.sweep(tiny, ws, ws_bytes, warmup=0, target_ms=0.0, min_reps=1, max_reps=1,
                cut_factor=0.0, dtype=dtype, pad_rows=pad)
    t0 = time.time()
    last_save = time.time()
    todo = [i for i in range(len(problems)) if (T[i] < 0).any()]
    log(f"sweep: {len(todo)} of {len(problems)} rows left, workspace {ws_bytes / 2**30:.2f} GiB", flush=True)
    for n_done, i in enumerate(todo):
        if time.time() - t0 > budget_s:
            log("sweep: time budget reached; rerun to resume", flush=True)
            break
        sub = T[i:i + 1].copy()
        ts = time.time()
        h.sweep([problems[i]], ws, ws_bytes, time_ns=sub, warmup=warmup, target_ms=target_ms,
                min_reps=min_reps, max_reps=max_reps, cut_factor=cut_factor, dtype=dtype,
                pad_rows=pad_rows)
        T[i] = sub[0]
        meta["seconds"] = meta.get("seconds", 0.0) + (time.time() - ts)
        if time.time() - last_save > 20 or n_done == len(todo) - 1:
            meta["finished"] = bool((T >= 0).all())
            save_table(out, T, problems, configs, meta)
            last_save = time.time()
        M, N, K, b, ta, tb = problems[i]
        best = int(T[i].min())
        log(f"sweep: row {i} ({M}x{N}x{K}x{b} {ta}{tb}) best {configs[int(T[i].argmin())]} "
            f"{2 * M * N * K * b / best / 1e3:.1f} TF, {time.time() - ts:.1f}s; "
            f"{int((T >= 0).all(axis=1).sum())}/{len(problems)} done", flush=True)
    meta["finished"] = bool((T >= 0).all())
    save_table(out, T, problems, configs, meta)
    return T


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--dtype", default="f32", choices=sorted(DTYPE_NAMES))
    s.add_argument("--set", default="sweep", choices=["sweep", "conv"])
    s.add_argument("--out", default=None)
    s.add_argument("--budget-s", type=float, default=900.0)
    s.add_argument("--limit", type=int, default=None)
    s.add_argument("--dense-rows", action="store_true",
                   help="operands with dense rows (default: rows padded to 16 bytes)")
    d = sub.add_parser("deploy")
    d.add_argument("--table", default=DEFAULT_TABLE)
    d.add_argument("--k", type=int, default=8)
    d.add_argument("--spec", default=DEPLOY_SPEC)
    d.add_argument("--out", default=DEPLOY_LIB)
    d.add_argument("--no-build", action="store_true")
    a = ap.parse_args(argv)
    if a.cmd == "sweep":
        run_sweep(a.out or table_path(a.dtype, a.set), a.budget_s, limit=a.limit,
                  dtype=DTYPE_NAMES[a.dtype], set_name=a.set, pad_rows=not a.dense_rows)
    elif a.cmd == "deploy":
        # choose the k kernels by GPU k-means over the training problems of the
        # measured table, record them, and build the library with only those
        import torch

        import synth
        from . import Handle, build
        T, P, C, meta = load_table(a.table)
        train, _ = synth.train_test_split()
        rows = synth.rows_of_shapes(train)
        h = Handle(0)
        ws_bytes = Handle.prune_workspace_bytes(len(rows), T.shape[1], a.k, 10)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        res = select_pruning(h, T[rows], a.k, synth.SEED, workspace=ws, ws_bytes=ws_bytes)
        chosen = res["chosen"]
        spec = dict(dtype="f32", k=a.k, chosen=chosen, kernels=[list(map(int, C[i])) for i in chosen],
                    config_ids=sorted({h.get_kernel(c)[1] for c in chosen}),
                    norm=res["norm_name"], train_ceiling=res["train_ceiling"], seed=synth.SEED,
                    n_init=10, max_iter=300, table=os.path.relpath(a.table, HERE),
                    device=meta.get("device"))
        os.makedirs(os.path.dirname(a.spec), exist_ok=True)
        with open(a.spec, "w") as f:
            json.dump(spec, f, indent=1)
        print("chosen", chosen, spec["kernels"], flush=True)
        if not a.no_build:
            build.build(f32_ids=spec["config_ids"], lp_ids=[], out=a.out, tag="deploy",
                        verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
