"""Profiling workload of the Toeplitz fast path: the N = 1e4 chain of Eq. (2)
(alpha = 1, w = ln N), 1024 trajectories, dt = 1e-4, FP32, 512 steps (two
launches of 256 steps after a one-launch warm-up), for rocprofv3 kernel traces
and counters."""
import math
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

if __name__ == "__main__":
    import torch
    import paper_2608_10075_amd as twa
    N, B, dt = 10000, 1024, 1e-4
    p = twa.build_pump_toeplitz(N, math.log(N), 1.0)
    twa.run(p, B, dt, 256, seed=0, precision="fp32", pump_path="toeplitz")
    torch.cuda.synchronize()
    t0 = time.time()
    r = twa.run(p, B, dt, 512, seed=0, precision="fp32", pump_path="toeplitz")
    torch.cuda.synchronize()
    print("toeplitz N=%d B=%d: %.3f ms per step (kernel %.3f)" % (N, B, 1e3 * (time.time() - t0) / 512,
                                                                 r.obs["kernel_ms"] / 512), flush=True)
