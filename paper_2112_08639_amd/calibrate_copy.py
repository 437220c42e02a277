"""Plain device copy of a known size, for calibrating hardware byte counters.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2112_08639_amd.calibrate_copy

copies a 512 MiB buffer once (torch's device copy kernel), so FETCH_SIZE and
WRITE_SIZE of that dispatch should read 512 MiB = 524288 KiB each; the ratio
scales the counters of the library's kernels.
"""

import torch

if __name__ == "__main__":
    n = 512 * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {x.numel() * 4 / 2**20:.0f} MiB")
