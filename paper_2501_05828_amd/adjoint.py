"""Differentiable simulation: scene parameters -> envelope image.

`simulate_envelope` is a torch.autograd.Function whose forward runs the
trace, pulse, delay-and-sum and envelope kernels and whose backward runs
their adjoints through the C ABI (ur_beamform_adjoint, ur_pulse_adjoint,
ur_trace_adjoint).  Gradients are the interior path-replay derivatives of
the estimator for the forward call's seed; with edge_terms the impedance and
sphere-centre gradients also take the direct hits' element-edge terms
(ur_trace_grad_edges).  include/ultraray.h says what each includes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding


class _EnvelopeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, amp, alpha, Z, sph_center, sim, seed, frozen_choice, edge_terms):
        sc = sim.w.scene
        mat = np.array(sc.materials, np.float64)
        mat[:, 0] = Z.detach().cpu().double().numpy()
        mat[:, 1] = alpha.detach().cpu().double().numpy()
        sph = np.array(sc.sph, np.float64).reshape(-1, 4)
        sph[:, :3] = sph_center.detach().cpu().double().numpy().reshape(-1, 3)
        sim.ctx.ur_scene_update(mat=mat, scat_amp=amp.detach().cpu().double().numpy(), sph=sph)
        sim.trace(seed)
        sim.beamform(bmode=False)
        ctx.sim, ctx.seed, ctx.frozen, ctx.edges = sim, seed, frozen_choice, edge_terms
        ctx.iq = sim.iq.clone()
        ctx.shapes = [(t.dtype, t.device, t.shape) for t in (amp, alpha, Z, sph_center)]
        return sim.env.clone()

    @staticmethod
    def backward(ctx, g_env):
        sim = ctx.sim
        dev = sim.dev
        need = ctx.needs_input_grad
        g_rf = torch.empty_like(sim.ch_rf)
        g_raw = torch.empty_like(sim.ch_raw)
        apod = binding.UR_APOD_HANN if sim.w.apod == "hann" else binding.UR_APOD_NONE
        sim.ctx.ur_beamform_adjoint(sim.w.grid, g_rf, iq=ctx.iq, g_env=g_env.contiguous().float(), apod=apod)
        sim.ctx.ur_pulse_adjoint(g_rf, g_raw)
        n_mat = len(sim.w.scene.materials)
        n_sph = len(sim.w.scene.sph)
        out = {
            "amp": torch.empty(len(sim.w.scene.scat), dtype=torch.float32, device=dev) if need[0] else None,
            "alpha": torch.empty(n_mat, dtype=torch.float64, device=dev) if need[1] else None,
            "Z": torch.empty(n_mat, dtype=torch.float64, device=dev) if need[2] else None,
            "sph": torch.empty((n_sph, 3), dtype=torch.float64, device=dev) if need[3] and n_sph else None,
        }
        if any(v is not None for v in out.values()):
            sim.ctx.ur_trace_adjoint(ctx.seed, g_raw, amp=out["amp"], alpha=out["alpha"], Z=out["Z"],
                                     sph_center=out["sph"], frozen_choice=ctx.frozen)
        if ctx.edges and (out["Z"] is not None or out["sph"] is not None):
            ez = torch.empty_like(out["Z"]) if out["Z"] is not None else None
            es = torch.empty_like(out["sph"]) if out["sph"] is not None else None
            sim.ctx.ur_trace_grad_edges(ctx.seed, g_raw, Z=ez, sph_center=es)
            if ez is not None:
                out["Z"] += ez
            if es is not None:
                out["sph"] += es
        grads = []
        for key, (dtype, device, shape) in zip(("amp", "alpha", "Z", "sph"), ctx.shapes):
            g = out[key]
            grads.append(None if g is None else g.to(dtype=dtype, device=device).reshape(shape))
        return (*grads, None, None, None, None)


def simulate_envelope(sim, amp, alpha, Z, sph_center, seed=None, frozen_choice=False, edge_terms=False):
    """Envelope image [nx][nz] of `sim`'s workload with the given scene
    parameters: scatterer amplitudes [n_scat], attenuation [n_mat] in
    dB/(cm MHz), impedances [n_mat] in MRayl and sphere centres [n_sph][3] in
    m (float tensors on any device).  Differentiable in all four.
    edge_terms (with the choice attached) adds the direct hits' element-edge
    terms to the impedance and sphere-centre gradients (linear arrays,
    uniform emission, smooth boundaries)."""
    seed = sim.w.seed if seed is None else seed
    if edge_terms and frozen_choice:
        raise ValueError("edge_terms estimate the derivative of the expected data: use frozen_choice=False")
    return _EnvelopeFn.apply(amp, alpha, Z, sph_center, sim, seed, frozen_choice, edge_terms)
