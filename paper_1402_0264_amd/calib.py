"""Calibration run for the HBM byte counters: a plain device-to-device copy
of a known size (256 MiB read, 256 MiB written per copy, 5 copies), so that
FETCH_SIZE and WRITE_SIZE as reported by the profiler can be scaled to
bytes (factor = known bytes / counter bytes per dispatch).

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1402_0264_amd.calib
"""
import sys

BYTES = 256 << 20


def main() -> int:
    import torch
    torch.cuda.set_device(0)
    src = torch.randint(0, 1 << 30, (BYTES // 4,), dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d bytes x 5" % BYTES, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
