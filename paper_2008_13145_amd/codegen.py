"""Build-time code generation of the kernel instantiation list.

The configuration space is defined here once; the generated C++ carries it
into the library (configuration table and launcher registry), so the id of a
configuration means the same thing everywhere.

FP32 space (the paper's R x A x C tile and work-group knobs of section 3,
re-designed for MFMA): bm, bn in {8,16,32,64,128}; t in {1,2,4,8} giving an
(8t) x (8t) wave block; bk in {8,16,32,64}; bm, bn multiples of 8t; 1..16
waves per work-group.  That is 164 configurations per layout and 656
instantiations over the four (transA, transB) layouts.

A "deploy" build instantiates only chosen ids (section 4: only the pruned
kernels ship in the library); ids keep their meaning, the rest are absent.
"""
from __future__ import annotations

import os

TILES = (8, 16, 32, 64, 128)
THREAD_TILES = (1, 2, 4, 8)
K_TILES = (8, 16, 32, 64)
LAYOUTS = ((0, 0), (0, 1), (1, 0), (1, 1))


def f32_configs():
    """Ordered list of (bm, bn, t, bk): the id is the position."""
    out = []
    for t in THREAD_TILES:
        wt = 8 * t
        for bm in TILES:
            for bn in TILES:
                if bm % wt or bn % wt:
                    continue
                waves = (bm * bn) // (wt * wt)
                if not 1 <= waves <= 16:
                    continue
                for bk in K_TILES:
                    out.append((bm, bn, t, bk))
    return out


def _chunks(seq, n):
    size = (len(seq) + n - 1) // n
    return [seq[i:i + size] for i in range(0, len(seq), size)]


def generate(out_dir: str, f32_ids=None, n_parts: int = 24):
    """Write the generated sources; return the list of .hip/.cpp paths."""
    os.makedirs(out_dir, exist_ok=True)
    cfgs = f32_configs()
    ids = list(range(len(cfgs))) if f32_ids is None else sorted(set(int(i) for i in f32_ids))
    insts = [(i, ta, tb) for i in ids for (ta, tb) in LAYOUTS]
    parts = _chunks(insts, max(1, min(n_parts, len(insts)))) if insts else []
    paths = []
    for p, chunk in enumerate(parts):
        lines = ['#include "gemm_f32.hpp"', '#include "registry.hpp"', "", "namespace kt {",
                 f"extern LaunchEntry f32_part{p}[] = {{"]
        for (i, ta, tb) in chunk:
            bm, bn, t, bk = cfgs[i]
            lines.append(f"  {{{i}, {ta}, {tb}, &launch_gemm_f32<{bm}, {bn}, {t}, {bk}, {ta}, {tb}>}},")
        lines += ["};", f"extern const int f32_part{p}_n = {len(chunk)};", "}  // namespace kt", ""]
        path = os.path.join(out_dir, f"f32_part{p}.hip")
        _write_if_changed(path, "\n".join(lines))
        paths.append(path)
    # configuration table + registry index
    lines = ['#include "registry.hpp"', "", "namespace kt {"]
    for p in range(len(parts)):
        lines.append(f"extern LaunchEntry f32_part{p}[];")
        lines.append(f"extern const int f32_part{p}_n;")
    lines.append("const ConfigDef f32_config_table[] = {")
    for (bm, bn, t, bk) in cfgs:
        lines.append(f"  {{{bm}, {bn}, {t}, {bk}}},")
    lines.append("};")
    lines.append(f"const int f32_config_count = {len(cfgs)};")
    lines.append("const PartRef f32_parts[] = {")
    for p in range(len(parts)):
        lines.append(f"  {{f32_part{p}, &f32_part{p}_n}},")
    if not parts:
        lines.append("  {nullptr, nullptr},")
    lines.append("};")
    lines.append(f"const int f32_part_count = {len(parts)};")
    lines += ["}  // namespace kt", ""]
    path = os.path.join(out_dir, "registry_gen.cpp")
    _write_if_changed(path, "\n".join(lines))
    paths.append(path)
    return paths


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as f:
        f.write(text)


if __name__ == "__main__":
    c = f32_configs()
    by_t = {t: sum(1 for x in c if x[2] == t) for t in THREAD_TILES}
    print(len(c), by_t)
