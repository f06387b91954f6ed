"""Plain device copy of a known size, for calibrating HBM byte counters.

``python -m paper_2211_01185_amd.calib`` copies a 256 MiB buffer into another
one ten times (torch's copy kernel).  Under ``rocprofv3 --pmc FETCH_SIZE`` (then
``WRITE_SIZE``) each dispatch should read (write) 262144 KiB; the ratio of the
counted value to that is the scale applied to the same counter measured on the
library's kernels.
"""
import torch

MIB = 1 << 20
BYTES = 256 * MIB


def main(reps: int = 10) -> None:
    src = torch.ones(BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {BYTES} bytes x {reps}", flush=True)


if __name__ == "__main__":
    main()
