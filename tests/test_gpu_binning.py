"""GPU: deterministic binning (ur_set_binning).

With deterministic binning the trace stages its records and bins them after
the trace with exact integer arithmetic, so the channel data are the same
bits on every call; they agree with the float-atomic binning to the
rounding of FP32 and with the FP64 oracle to the parity tolerance of the
channel data (1e-4 relative L2).
"""
import numpy as np
import pytest

from paper_2501_05828_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.mark.parametrize("binning", [scenes.NEAREST, scenes.LINEAR])
def test_deterministic_binning(oracle, torch_gpu, binning):
    import dataclasses
    from paper_2501_05828_amd.sim import Simulator
    w = scenes.tiny(rays_per_element=1024)
    # wide receive cones: many records share each bin, so the order of
    # arrival changes the float-atomic sums
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, binning=binning, alpha_m=np.deg2rad(10.0),
                                                       alpha_c=np.deg2rad(45.0)))
    s = Simulator(w)
    s.trace(pulse=False)
    atomic = s.ch_raw.clone()
    s.ctx.ur_set_binning(True, 1 << 20)
    try:
        st = s.trace(pulse=False, stats=True)
        d1 = s.ch_raw.clone()
        s.trace(pulse=False)
        d2 = s.ch_raw.clone()
    finally:
        s.ctx.ur_set_binning(False)
    ref, _ = oracle.trace(w)
    a, b, o = atomic.cpu().double().numpy(), d1.cpu().double().numpy(), ref
    rel_atomic = np.linalg.norm(b - a) / np.linalg.norm(a)
    rel_oracle = np.linalg.norm(b - o) / np.linalg.norm(o)
    print(f"[binning] records {st['records']}, deterministic vs atomic {rel_atomic:.2e}, vs oracle {rel_oracle:.2e}",
          flush=True)
    assert st["records"] > 500
    assert torch_gpu.equal(d1, d2)
    assert rel_atomic <= 1e-6
    assert rel_oracle <= 1e-4


def test_deterministic_binning_capacity(torch_gpu):
    from paper_2501_05828_amd.binding import URError
    from paper_2501_05828_amd.sim import Simulator
    s = Simulator(scenes.tiny(rays_per_element=1024))
    s.ctx.ur_set_binning(True, 10)
    with pytest.raises(URError, match="CAPACITY"):
        s.trace(pulse=False)
    s.ctx.ur_set_binning(False)
    s.trace(pulse=False)
    assert s.ctx.lib.ur_set_binning(s.ctx.h, 2, 10) == -1   # UR_ERR_INVALID_ARG: mode not 0 or 1
    with pytest.raises(URError, match="INVALID_ARG"):
        s.ctx.ur_set_binning(True, 0)


def test_deterministic_binning_with_sampling_overflow(oracle, torch_gpu):
    """A transducer-sampling queue far too small: each range is traced again
    with inline secondary rays, whose records are staged like the others;
    the channel data still match the oracle and repeat bit for bit."""
    import dataclasses
    import math
    from paper_2501_05828_amd.sim import Simulator
    w = scenes.tiny(rays_per_element=512)
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45)))
    s = Simulator(w)
    s.ctx.ur_set_limits(4096, 7)
    s.ctx.ur_set_binning(True, 1 << 20)
    try:
        s.trace(pulse=False)
        d1 = s.ch_raw.clone()
        s.trace(pulse=False)
        d2 = s.ch_raw.clone()
    finally:
        s.ctx.ur_set_binning(False)
    ref, _ = oracle.trace(w)
    b = d1.cpu().double().numpy()
    rel = np.linalg.norm(b - ref) / np.linalg.norm(ref)
    print(f"[binning] overflow re-trace, deterministic vs oracle {rel:.2e}", flush=True)
    assert torch_gpu.equal(d1, d2)
    assert rel <= 1e-4


def test_deterministic_binning_across_admitted_launches(oracle, torch_gpu):
    """A segment budget that splits the trace into several launches: the
    records of every launch are staged and binned once after the last."""
    import dataclasses
    import math
    from paper_2501_05828_amd.sim import Simulator
    w = scenes.tiny(rays_per_element=1024)
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45)))
    s = Simulator(w)
    s.ctx.ur_set_binning(True, 1 << 20)
    try:
        s.trace(pulse=False)
        one = s.ch_raw.clone()
        s.ctx.ur_set_segment_queue(20_000)
        s.trace(pulse=False)
        launches = s.ctx.ur_last_trace_kernels_ms()[3]
        split = s.ch_raw.clone()
    finally:
        s.ctx.ur_set_binning(False)
        s.ctx.ur_set_segment_queue(0)
    ref, _ = oracle.trace(w)
    rel = np.linalg.norm(split.cpu().double().numpy() - ref) / np.linalg.norm(ref)
    print(f"[binning] {launches} launches, deterministic vs oracle {rel:.2e}", flush=True)
    assert launches >= 2
    assert torch_gpu.equal(one, split)
    assert rel <= 1e-4
