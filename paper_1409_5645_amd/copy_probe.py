"""Calibration of HBM traffic counters: a plain device copy of a known size.

Run under `rocprofv3 --pmc FETCH_SIZE` (and, in a run of its own,
`--pmc WRITE_SIZE`): every copy dispatch reads and writes exactly `nbytes`, so
the counter value divided by the known size is the factor by which the same
counter over-reports (or under-reports) bytes for other kernels on this GPU.

    python -m paper_1409_5645_amd.copy_probe [nbytes]
"""
from __future__ import annotations

import json
import sys


def main() -> None:
    import torch
    nbytes = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    reps = 5
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "dispatches": reps, "check": float(b[-1])}), flush=True)


if __name__ == "__main__":
    main()
