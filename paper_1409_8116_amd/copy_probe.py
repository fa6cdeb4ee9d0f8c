"""Plain device copy of a known size (HBM counter calibration for profiles).

Run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE: the counters this copy
reports, divided by its known bytes, give the scale factor applied to the
solver kernels' counters.
"""
import sys

import torch


def main():
    nbytes = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x3", flush=True)


if __name__ == "__main__":
    main()
