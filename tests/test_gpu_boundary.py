"""GPU: the direct-hit edge terms of the gradient (ur_trace_grad_edges).

The terms that the interior adjoint leaves out where a direct hit's landing
point crosses an element edge, an end of the aperture or an elevation edge,
integrated along the emission origin of every path family, against the
FP64 oracle's or_trace_grad_edges (pinned on the CPU by
tests/test_oracle_edges.py) on the same paths and scan.  Both sides locate
the same crossings by the same bisections and Newton steps, so the sums
agree to the rounding of the replays.
"""
import dataclasses

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _case():
    import test_oracle_edges as T
    w = T._workload(128)
    return w, T._adjoint(w.acq, 5).astype(np.float32)


def test_edge_terms_match_oracle(oracle, torch_gpu):
    from paper_2501_05828_amd.sim import Simulator
    torch = torch_gpu
    w, g = _case()
    nm, ns = len(w.scene.materials), len(w.scene.sph)
    ref = oracle.trace_grad_edges(w, g.astype(np.float64), n_scan=16)
    s = Simulator(w)
    Z = torch.empty(nm, dtype=torch.float64, device="cuda")
    cen = torch.empty((ns, 3), dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_grad_edges(w.seed, torch.from_numpy(g).cuda(), Z=Z, sph_center=cen, n_scan=16)
    got = dict(z=Z.cpu().numpy(), sph=cen.cpu().numpy())
    for key in ("z", "sph"):
        a, b = got[key].ravel(), ref[key].ravel()
        scale = np.abs(b).max()
        print(f"[edges-gpu] {key}: oracle {b} gpu {a} max err {np.abs(a - b).max():.3e}", flush=True)
        assert scale > 0.0
        assert np.array_equal(a[b == 0.0], b[b == 0.0])
        assert np.abs(a - b).max() <= 1e-6 * scale


def test_edge_terms_refuse_convex_arrays(torch_gpu):
    from paper_2501_05828_amd.binding import URError
    from paper_2501_05828_amd.sim import Simulator
    torch = torch_gpu
    w, g = _case()
    w = scenes.convex_probe(w, 20e-3)
    s = Simulator(w)
    Z = torch.empty(len(w.scene.materials), dtype=torch.float64, device="cuda")
    with pytest.raises(URError):
        s.ctx.ur_trace_grad_edges(w.seed, torch.from_numpy(g).cuda(), Z=Z)
