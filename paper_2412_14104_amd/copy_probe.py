"""Plain device copy of a known size, used to calibrate the HBM byte counters
(FETCH_SIZE / WRITE_SIZE) of rocprofv3 against algorithmic bytes.

    python paper_2412_14104_amd/copy_probe.py [MiB]
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d MiB x 3 (read %d MiB + write %d MiB per copy)" % (mib, mib, mib), flush=True)


if __name__ == "__main__":
    main()
