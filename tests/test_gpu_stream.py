"""The measured read-stream bandwidth the HBM-bound kernels are compared with.

Properties that hold on any MI355X: the rate of a 1 GiB read (four times the
last-level cache) is positive and below the 8 TB/s published peak; the same
call on a buffer with a ragged tail (not a multiple of the grid's stride)
returns normally; re-reading a buffer that fits the last-level cache is not
slower than streaming one four times its size (10 % slack for run-to-run
noise).  The measured exponential rate is positive and at most the ceiling
that the unit counts and the clock give (256 CUs x 4 SIMDs x 64 lanes, one
v_exp_f32 per 8 cycles per wave, 2.4 GHz), with 5 % slack.
"""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_read_bandwidth_below_peak(torch_gpu):
    torch = torch_gpu
    from paper_2605_30267_amd import accsk
    buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    gbps = accsk.read_bandwidth(buf, reps=5)
    print("read stream GB/s", gbps, flush=True)
    assert math.isfinite(gbps) and 1000.0 < gbps < 8000.0
    tail = torch.ones((1 << 20) + 12, dtype=torch.float32, device="cuda")
    assert accsk.read_bandwidth(tail, reps=2) > 0
    small = accsk.read_bandwidth(buf[: 1 << 26], reps=20)
    print("re-read of 256 MiB GB/s", small, flush=True)
    assert small >= 0.9 * gbps


def test_exp_rate_below_ceiling(torch_gpu):
    from paper_2605_30267_amd import accsk
    rate = accsk.exp_rate(reps=3)
    print("v_exp_f32 per second", rate, flush=True)
    ceiling = 256 * 4 * 64 / 8 * 2.4e9
    assert math.isfinite(rate) and 0.25 * ceiling < rate < 1.05 * ceiling
