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

Kernels: the configurations of a dtype (ids 0 .. n-1) are followed by its
split-K variants (ids n, n+1, ...), the kernel type section 3 names for deep,
under-filled products: a base configuration run over S slices of K plus a
reduction.  A variant adds no code (it reuses its base's instantiation), so a
deploy build that keeps the base keeps its variants.
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


LP_TILES = (32, 64, 128, 256)
LP_THREAD_TILES = (4, 8, 16)
BF16_K_TILES = (32, 64, 128)     # multiples of the BF16 MFMA depth (16)
FP8_K_TILES = (64, 128, 256)     # multiples of the FP8 MFMA depth (64)


def _lp_configs(k_tiles, elem_bytes):
    """Ordered (bm, bn, t, bk) list of a low-precision family: wave blocks of
    32x32 (t = 4), 64x64 (t = 8) or 128x128 (t = 16) MFMA outputs, 1..16
    waves, and double-buffered LDS stages (rows padded by 16 bytes) within
    160 KiB."""
    out = []
    for t in LP_THREAD_TILES:
        wt = 8 * t
        for bm in LP_TILES:
            for bn in LP_TILES:
                if bm % wt or bn % wt:
                    continue
                waves = (bm * bn) // (wt * wt)
                if not 1 <= waves <= 16:
                    continue
                for bk in k_tiles:
                    if 2 * (bm + bn) * (bk * elem_bytes + 16) > 160 * 1024:
                        continue
                    out.append((bm, bn, t, bk))
    return out


# 16x16 wave blocks (t = 2, the 16x16 MFMAs) for small and skinny problems,
# appended after the larger blocks so the earlier ids keep their meaning; the
# FP8 16x16 MFMA is 128 deep.
SMALL_TILES = (16, 32, 64, 128, 256)
BF16_SMALL_K_TILES = (32, 64)
FP8_SMALL_K_TILES = (128,)


def _lp_small_configs(k_tiles):
    out = []
    for bm in SMALL_TILES:
        for bn in SMALL_TILES:
            waves = (bm // 16) * (bn // 16)
            if not 1 <= waves <= 16:
                continue
            for bk in k_tiles:
                out.append((bm, bn, 2, bk))
    return out


def bf16_configs():
    return _lp_configs(BF16_K_TILES, 2) + _lp_small_configs(BF16_SMALL_K_TILES)


def fp8_configs():
    return _lp_configs(FP8_K_TILES, 1) + _lp_small_configs(FP8_SMALL_K_TILES)


SPLIT_TILES = ((16, 16), (32, 32), (64, 64), (128, 128), (16, 128), (128, 16))
SPLIT_SLICES = (2, 4, 8, 16)


def split_variants(cfgs):
    """Split-K variants of a configuration list, as (base id, slices): for
    each work-group tile in SPLIT_TILES (square tiles, then the two skinny
    ones for products with a single row or column block, such as a
    matrix-vector product), the configuration with the deepest K tile and,
    among those, the most waves (smallest t), run over 2, 4, 8 and 16
    slices.  New tiles go at the end, so earlier kernel ids keep their
    meaning."""
    out = []
    for (tm, tn) in SPLIT_TILES:
        cand = [(i, c) for i, c in enumerate(cfgs) if c[0] == tm and c[1] == tn]
        if not cand:
            continue
        base = min(cand, key=lambda ic: (-ic[1][3], ic[1][2], ic[0]))[0]
        out += [(base, s) for s in SPLIT_SLICES]
    return out


def kernels(cfgs):
    """(bm, bn, t, bk, slices) per kernel id: configurations, then split-K variants."""
    return [tuple(c) + (1,) for c in cfgs] + [tuple(cfgs[b]) + (s,) for (b, s) in split_variants(cfgs)]


DTYPES = (  # (name, config list, launcher template)
    ("f32", f32_configs, "launch_gemm_f32<{bm}, {bn}, {t}, {bk}, {ta}, {tb}>", "gemm_f32_dma.hpp"),
    ("bf16", bf16_configs, "launch_gemm_lp<2, {bm}, {bn}, {t}, {bk}, {ta}, {tb}>", "gemm_lp_dma.hpp"),
    ("fp8", fp8_configs, "launch_gemm_lp<1, {bm}, {bn}, {t}, {bk}, {ta}, {tb}>", "gemm_lp_dma.hpp"),
)


def _chunks(seq, n):
    """Round-robin split (neighbouring configurations cost alike to compile,
    so interleaving balances the parallel build)."""
    return [seq[i::n] for i in range(n) if seq[i::n]]


def generate(out_dir: str, f32_ids=None, lp_ids=None, n_parts: int = 24, lp_parts: int = 12):
    """Write the generated sources; return the list of .hip/.cpp paths.
    f32_ids / lp_ids restrict the instantiated configurations (deploy build);
    None means all."""
    os.makedirs(out_dir, exist_ok=True)
    paths = []
    reg = ['#include "registry.hpp"', "", "namespace kt {"]
    tables = []
    for (name, cfg_fn, tmpl, header) in DTYPES:
        cfgs = cfg_fn()
        sel = f32_ids if name == "f32" else lp_ids
        ids = list(range(len(cfgs))) if sel is None else sorted(set(int(i) for i in sel))
        insts = [(i, ta, tb) for i in ids for (ta, tb) in LAYOUTS]
        nparts = n_parts if name == "f32" else lp_parts
        parts = _chunks(insts, max(1, min(nparts, len(insts)))) if insts else []
        for p, chunk in enumerate(parts):
            lines = [f'#include "{header}"', '#include "registry.hpp"', "", "namespace kt {",
                     f"extern LaunchEntry {name}_part{p}[] = {{"]
            for (i, ta, tb) in chunk:
                bm, bn, t, bk = cfgs[i]
                fn = tmpl.format(bm=bm, bn=bn, t=t, bk=bk, ta=ta, tb=tb)
                lines.append(f"  {{{i}, {ta}, {tb}, &{fn}}},")
            lines += ["};", f"extern const int {name}_part{p}_n = {len(chunk)};",
                      "}  // namespace kt", ""]
            path = os.path.join(out_dir, f"{name}_part{p}.hip")
            _write_if_changed(path, "\n".join(lines))
            paths.append(path)
        for p in range(len(parts)):
            reg.append(f"extern LaunchEntry {name}_part{p}[];")
            reg.append(f"extern const int {name}_part{p}_n;")
        reg.append(f"static const ConfigDef {name}_configs[] = {{")
        for (bm, bn, t, bk) in cfgs:
            reg.append(f"  {{{bm}, {bn}, {t}, {bk}}},")
        reg.append("};")
        splits = split_variants(cfgs)
        reg.append(f"static const SplitDef {name}_splits[] = {{")
        for (b, sl) in splits:
            reg.append(f"  {{{b}, {sl}}},")
        reg.append("};")
        reg.append(f"static const PartRef {name}_parts[] = {{")
        for p in range(len(parts)):
            reg.append(f"  {{{name}_part{p}, &{name}_part{p}_n}},")
        if not parts:
            reg.append("  {nullptr, nullptr},")
        reg.append("};")
        tables.append(f"  {{{name}_configs, {len(cfgs)}, {name}_splits, {len(splits)}, "
                      f"{name}_parts, {len(parts)}}},")
    reg.append("const DtypeRegistry dtype_registry[3] = {")
    reg += tables
    reg.append("};")
    reg += ["}  // namespace kt", ""]
    path = os.path.join(out_dir, "registry_gen.cpp")
    _write_if_changed(path, "\n".join(reg))
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
    print("f32", len(c), by_t)
    print("bf16", len(bf16_configs()), "fp8", len(fp8_configs()))
    for name, fn in (("f32", f32_configs), ("bf16", bf16_configs), ("fp8", fp8_configs)):
        cf = fn()
        print(name, "split-K bases", sorted({cf[b] for (b, _) in split_variants(cf)}))
