"""Calibration kernel for HBM byte counters: one plain device copy of a known
size (1 GiB read, 1 GiB written), run under rocprofv3 --pmc FETCH_SIZE /
WRITE_SIZE to obtain the scale between counter readings and bytes moved."""
import torch

if __name__ == "__main__":
    n = 1 << 28                      # 2^28 float32 = 1 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes" % (4 * n), flush=True)
