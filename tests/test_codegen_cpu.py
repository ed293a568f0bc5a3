"""Generated-code checks of the LDS-DMA pipelines (gfx950 assembly of our own
sources, compiled here on the CPU).

The stage pipeline keeps the next stage's LDS DMA in flight while the current
stage's fragments are read and multiplied; its own waits (vmcnt + barrier at
the top of each stage) order every transfer.  A compiler-inserted vmcnt wait
between a DMA issue and the following LDS fragment reads would wait for that
next stage too and serialize transfer and MFMAs.  These tests compile one
instantiation per pipeline and check that no such wait is generated."""
import os
import re
import shutil
import subprocess

import pytest


def _hipcc():
    from paper_2008_13145_amd import build
    return build.HIPCC if os.path.exists(build.HIPCC) else shutil.which("hipcc")


def _device_asm(tmp_path, header, inst):
    from paper_2008_13145_amd import build
    hipcc = _hipcc()
    if not hipcc:
        pytest.skip("hipcc not available")
    src = tmp_path / "inst.hip"
    src.write_text(f'#include "{header}"\nnamespace kt {{\n{inst}\n}}\n')
    out = tmp_path / "inst.s"
    cmd = [hipcc] + build.CXXFLAGS + ["-x", "hip", "-I", build.CSRC, "-I", build.INCLUDE,
                                      "--offload-device-only", "-S", str(src), "-o", str(out)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
    return out.read_text()


def _guarded_lds_reads(asm):
    """Compiler-generated vmcnt waits (outside inline-asm blocks) that sit
    between an LDS DMA issue and the next LDS read, per kernel."""
    found, cur, seen_dma, pending, in_asm = {}, None, False, False, False
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur, seen_dma, pending, in_asm = m.group(1), False, False, False
            found[cur] = 0
            continue
        if cur is None:
            continue
        if "ASMSTART" in line:
            in_asm, pending = True, False
            continue
        if "ASMEND" in line:
            in_asm = False
            continue
        if in_asm:
            if "global_load_lds" in line:
                seen_dma = True
            continue
        if "global_load_lds" in line:
            seen_dma = True
        elif "s_waitcnt" in line and "vmcnt" in line and seen_dma:
            pending = True
        elif "global_store" in line or "global_load_dword " in line or "scratch_load" in line:
            pending = False
        elif "ds_read" in line and pending:
            found[cur] += 1
            pending = False
    return found


def test_low_precision_dma_has_no_compiler_wait_before_fragment_reads(tmp_path):
    # B stored N-contiguous: its fragments come from the LDS transpose reads
    asm = _device_asm(tmp_path, "gemm_lp_dma.hpp",
                      "template __global__ void gemm_lp_dma_kernel<2, 128, 128, 8, 64, 0, 0>"
                      "(GemmArgs);\n"
                      "template __global__ void gemm_lp_dma_kernel<1, 256, 256, 8, 128, 1, 0>"
                      "(GemmArgs);")
    found = _guarded_lds_reads(asm)
    assert len(found) == 2 and "global_load_lds_dwordx4" in asm
    assert all(v == 0 for v in found.values()), found


def test_fp32_dma_has_no_compiler_wait_before_fragment_reads(tmp_path):
    asm = _device_asm(tmp_path, "gemm_f32_dma.hpp",
                      "template __global__ void gemm_f32_dma_kernel<128, 128, 4, 32, 1, 0>"
                      "(GemmArgs);\n"
                      "template __global__ void gemm_f32_dma_kernel<64, 64, 2, 32, 0, 1>"
                      "(GemmArgs);")
    found = _guarded_lds_reads(asm)
    assert len(found) == 2 and "global_load_lds_dwordx4" in asm
    assert all(v == 0 for v in found.values()), found
