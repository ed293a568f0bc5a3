"""Known-traffic kernel for calibrating HBM byte counters.

Runs the BF16 conversion kernel (reads 4 bytes and writes 2 bytes per
element, each exactly once) on a buffer far larger than the caches, so that
rocprofv3's FETCH_SIZE and WRITE_SIZE for its dispatches can be compared with
the known byte counts:

    rocprofv3 --pmc FETCH_SIZE -d OUT -o calib -- python3 -m paper_2008_13145_amd.calibrate
    rocprofv3 --pmc WRITE_SIZE -d OUT -o calib -- python3 -m paper_2008_13145_amd.calibrate

Prints the element count and the expected bytes per dispatch.
"""
from __future__ import annotations

import argparse
import json


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch

    import paper_2008_13145_amd as kt
    n = 1 << a.log2n
    h = kt.Handle(0)
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    h.fill_uniform(x, n, 1)
    y = torch.empty(n, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    for _ in range(a.reps):
        h.convert_bf16(x, n, y)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "cvt_bf16_kernel", "elements": n, "fetch_bytes": 4 * n,
                      "write_bytes": 2 * n, "dispatches": a.reps}))


if __name__ == "__main__":
    main()
