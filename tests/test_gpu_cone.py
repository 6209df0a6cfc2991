"""Cone-restricted element choice of transducer sampling (UR_ELEMENT_CONE) on
the GPU against the FP64 oracle, and in the adjoint's replay."""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

pytestmark = pytest.mark.gpu

EXACT = ["rays", "segments", "reflect", "transmit", "tir", "nee_cast", "nee_blocked", "direct_hits", "records",
         "dropped", "edge_band", "term_box", "term_bounce", "term_time", "term_path", "media_mismatch", "term_rough"]


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (nb if nb > 0 else 1.0)


def _cone(w, am=4.0, ac=10.0, **kw):
    return dataclasses.replace(w, acq=dataclasses.replace(w.acq, alpha_m=math.radians(am), alpha_c=math.radians(ac),
                                                          element_choice=scenes.ELEMENT_CONE, **kw))


def _compare(oracle, w, stride=1, label=""):
    from paper_2501_05828_amd.sim import Simulator
    print(f"[cone] {label}", flush=True)
    s = Simulator(w)
    st = s.trace(stats=True, ray_stride=stride, pulse=False)
    g = s.ch_raw.cpu().numpy().astype(np.float64)
    ref, ost = oracle.trace(w, ray_stride=stride)
    for k in EXACT:
        assert st[k] == ost[k], (label, k, st[k], ost[k])
    assert st["scatter_events"] - st["nee_zero"] == ost["scatter_events"] - ost["nee_zero"]
    err = rel_l2(g, ref)
    print(f"[cone] {label} records={ost['records']} nee_cast={ost['nee_cast']} rel_l2={err:.3e}", flush=True)
    assert np.array_equal(g != 0, ref != 0) and err <= 1e-4
    return st, ost


def test_cone_tiny(torch_gpu, oracle):
    st, ost = _compare(oracle, _cone(scenes.tiny()), label="tiny")
    assert ost["nee_cast"] > 500


def test_cone_tiny_paper_angles(torch_gpu, oracle):
    """alpha_m = alpha_c = 2 degrees (Sec. 4): a hard cut."""
    _compare(oracle, _cone(scenes.tiny(), 2.0, 2.0), label="tiny-2deg")


def test_cone_bone_sampled(torch_gpu, oracle):
    _compare(oracle, _cone(scenes.bone(), 2.0, 2.0), stride=2000, label="bone-sampled")


def test_cone_explicit_rays_same_events(torch_gpu, oracle):
    w = _cone(scenes.tiny())
    rng = np.random.default_rng(23)
    rays = []
    for r in range(3000):
        o = [rng.uniform(-9, 9) * 1e-3, rng.uniform(-2, 2) * 1e-3, 0.0]
        th, ph = math.acos(rng.uniform(0.3, 1.0)), rng.uniform(0, 2 * math.pi)
        d = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
        rays.append(dict(o=o, d=d, w=1.0, t=1e-7 * r, ray=r, elem=r % 64))
    from paper_2501_05828_amd.sim import Simulator
    s = Simulator(w)
    ev_g, n_g = s.ctx.ur_trace_rays(w.seed, rays, cap=200000)
    ev_o, _, _ = oracle.trace_rays(w, rays, cap=200000)
    assert n_g == len(ev_o)
    key = lambda e: (e["tx"], e["kind"], e["seg"], e["id"], e["elem"], round(e["t"] * 1e12))
    ev_g, ev_o = sorted(ev_g, key=key), sorted(ev_o, key=key)
    n_sc = 0
    for a, b in zip(ev_g, ev_o):
        assert (a["kind"], a["seg"], a["id"], a["elem"]) == (b["kind"], b["seg"], b["id"], b["elem"])
        assert abs(a["t"] - b["t"]) <= 1e-15 + 1e-12 * abs(b["t"])
        assert abs(a["value"] - b["value"]) <= 1e-5 * abs(b["value"]) + 1e-300
        n_sc += a["kind"] == "scatter"
    assert n_sc > 10


def test_cone_adjoint_value_and_amplitude_gradient(torch_gpu, oracle):
    """The replay in cone mode: its value equals the forward channel data
    weighted by g, and the amplitude gradient along a direction equals the
    oracle's central difference."""
    torch = torch_gpu
    from paper_2501_05828_amd.sim import Simulator
    w = _cone(scenes.tiny(rays_per_element=1024), 4.0, 10.0, binning=scenes.LINEAR)
    rng = np.random.default_rng(31)
    g = rng.normal(size=(1, w.acq.n_elements, w.acq.n_samples)).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    s = Simulator(w)
    s.trace(pulse=False)
    j_fwd = float((s.ch_raw.double() * gt.double()).sum())
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    amp = torch.empty(len(w.scene.scat), device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, amp=amp, value=v)
    assert abs(v.item() - j_fwd) <= 1e-5 * abs(j_fwd) + 1e-12
    ga = amp.double().cpu().numpy()
    d = rng.normal(size=len(ga))
    a0 = w.scene.scat[:, 3].copy()

    def J(h):
        ww = dataclasses.replace(w, scene=dataclasses.replace(
            w.scene, scat=np.column_stack([w.scene.scat[:, :3], a0 + h * d])))
        ch, _ = oracle.trace(ww)
        return float((ch * g).sum())

    fd = (J(1.0) - J(-1.0)) / 2.0        # linear in the amplitudes: exact difference
    assert abs(float(ga @ d) - fd) <= 1e-5 * np.linalg.norm(ga) * np.linalg.norm(d) + 1e-6 * abs(fd)
