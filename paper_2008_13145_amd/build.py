"""Compile libkt.so for gfx950 with hipcc (in-tree, no JIT cache).

``build()`` generates the instantiation list (``codegen.py``), compiles every
translation unit in parallel and links ``paper_2008_13145_amd/libkt.so``.
``build(f32_ids=[...], out=...)`` makes a deploy build that contains only the
chosen configurations (the pruned kernel set of section 4 of the paper).

Run as ``python -m paper_2008_13145_amd.build [--jobs N]``.
"""
from __future__ import annotations

import argparse
import glob
import os
import shutil
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(HERE, "libkt.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src, obj, verbose):
    cmd = [HIPCC] + CXXFLAGS + ["-x", "hip", "-I", CSRC, "-I", INCLUDE, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 feature; that warning is harmless
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if verbose:
        print(f"  {os.path.basename(src)}: {time.time() - t0:.1f}s", flush=True)
    return obj


def _local_includes(path, seen):
    """Files reached through #include "..." from path (searched next to the
    including file, then in csrc/ and include/)."""
    import re
    for line in open(path):
        m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
        if not m:
            continue
        for base in (os.path.dirname(path), CSRC, INCLUDE):
            cand = os.path.normpath(os.path.join(base, m.group(1)))
            if os.path.exists(cand):
                if cand not in seen:
                    seen.add(cand)
                    _local_includes(cand, seen)
                break
    return seen


def _up_to_date(src, obj):
    """True when obj is newer than its source and every header it includes."""
    if not os.path.exists(obj):
        return False
    deps = [src] + sorted(_local_includes(src, set()))
    return os.path.getmtime(obj) > max(os.path.getmtime(d) for d in deps)


def build(jobs: int | None = None, f32_ids=None, lp_ids=None, out: str = LIB,
          verbose: bool = False, tag: str = "full", incremental: bool = False) -> str:
    """Compile and link; returns the path of the shared library.  With
    incremental=True, objects newer than their source and every header are
    reused (a development shortcut; the default recompiles everything)."""
    from . import codegen
    bdir = os.path.join(HERE, "_build", tag)
    gdir = os.path.join(bdir, "gen")
    odir = os.path.join(bdir, "obj")
    os.makedirs(odir, exist_ok=True)
    gen = codegen.generate(gdir, f32_ids=f32_ids, lp_ids=lp_ids)
    srcs = _sources() + gen
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = [os.path.join(odir, os.path.basename(s) + ".o") for s in srcs]
    t0 = time.time()
    todo = [(so, o) for so, o in zip(srcs, objs) if not (incremental and _up_to_date(so, o))]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), todo))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} ({os.path.getsize(out)} bytes) in {time.time() - t0:.1f}s", flush=True)
    return out


def build_deploy(jobs: int | None = None, verbose: bool = False):
    """Deploy build from the recorded k-means choice (data/deploy_f32.json):
    only the chosen FP32 configurations, in all four layouts.  Returns the
    library path, or None when no choice has been recorded."""
    import json
    spec_path = os.path.join(HERE, "data", "deploy_f32.json")
    if not os.path.exists(spec_path):
        return None
    spec = json.load(open(spec_path))
    # the configurations of the chosen kernels (a split-K variant runs its base's code)
    ids = spec.get("config_ids", spec["chosen"])
    return build(jobs=jobs, f32_ids=ids, lp_ids=[],
                 out=os.path.join(HERE, "libkt_deploy.so"), verbose=verbose, tag="deploy")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--ids", type=str, default=None, help="comma-separated FP32 config ids (deploy build)")
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--deploy", action="store_true", help="also build the recorded deploy library")
    ap.add_argument("--incremental", action="store_true",
                    help="reuse objects newer than their sources and headers")
    a = ap.parse_args(argv)
    ids = None if a.ids is None else [int(x) for x in a.ids.split(",") if x]
    out = a.out or (LIB if ids is None else os.path.join(HERE, "libkt_deploy.so"))
    build(jobs=a.jobs, f32_ids=ids, lp_ids=None if ids is None else [], out=out, verbose=True,
          tag="full" if ids is None else "deploy", incremental=a.incremental)
    if a.deploy and ids is None:
        build_deploy(jobs=a.jobs, verbose=True)


if __name__ == "__main__":
    main()
