"""Benchmark of the full-path ultrasound simulation on one MI355X.

A step is one pass of the hot path over one acquisition of the bone-phantom
workload (128 elements, 11 plane waves -10..10 deg, 1e7 rays per transmit,
8 bounces, 60k-triangle tube, 3 slabs, 50k scatterers, 4096 samples): trace
and bin every ray, pulse-shape the channel data, delay-and-sum to a 512x512
compounded image, envelope and log compression.  Inputs are resident on the
GPU before timing starts; each step draws a fresh Philox key.

Prints one JSON line.  The roofline entry is for the extend kernel (the
dominant kernel of the trace): algorithmic FLOPs (per-unit costs below x
unit counts from an instrumented pass over the same workload) divided by its
duration, both per frame; a frame launches the kernel once per launch, so
this equals the average FLOPs per launch over the average launch
duration.  Durations come from HIP events that the library records on the
stream it launches on.  The scatter kernel is reported beside it.  The CPU
baseline is the FP64 oracle timed on a bounded, evenly strided sample of the
same rays.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "traced rays/s + DAS frames/s; channel MSE at equal GPU time, learned vs uniform"
PEAK_FP32 = 157.3e12      # MI355X vector FP32 (256 CU x 2.4 GHz x 256 FLOP/clk with packed FMA)
PEAK_FP64 = 78.6e12       # MI355X vector FP64 (256 CU x 2.4 GHz x 128 FLOP/clk)
PEAK_HBM = 8.0e12
N_CU = 256
CLOCK_HZ = 2.4e9

# Algorithmic FLOPs per counted unit (add/sub/mul = 1, fma = 2,
# div/sqrt/exp/acos = 1; compares, min/max and integer RNG work are not
# counted).  Only the part of each test that always executes is counted.
# Extend kernel (emission, closest hits, interfaces):
FP32_PER_NODE = 48          # four-wide node: four slab tests of 6 fma (child planes from 8-bit offsets)
FP64_PER_TRI_TEST = 24      # Moller-Trumbore up to the first barycentric test
FP64_PER_SEGMENT = 16       # box exit (6) + transport (10)
FP64_PER_PLANE = 12         # per plane per segment
FP64_PER_SPHERE = 20        # per sphere per segment
FP64_PER_INTERFACE = 60     # normal, Eqs. 7-11, new direction, renormalisation
FP64_PER_RAY = 40           # emission: origin, hemisphere map, weight
# Scatter kernel (captures):
FP64_PER_CELL = 4           # grid walk step: next crossing (fma) + advance
FP32_PER_SCAT_TEST = 16     # FP32 prefilter: offset (3), projection, perpendicular and its length (fma)
FP64_PER_EVENT = 33         # exact capture test (8) + projection point, element geometry, directivity (25)


def extend_flops(st, n_pln, n_sph):
    """FP32 and FP64 FLOPs of the extend kernel for one frame."""
    f32 = FP32_PER_NODE * st["tri_nodes"]
    f64 = (FP64_PER_TRI_TEST * st["tri_tests"]
           + st["segments"] * (FP64_PER_SEGMENT + FP64_PER_PLANE * n_pln + FP64_PER_SPHERE * n_sph)
           + FP64_PER_INTERFACE * (st["reflect"] + st["transmit"] + st["tir"])
           + FP64_PER_RAY * st["rays"])
    return float(f32), float(f64)


def scatter_flops(st):
    """FP32 and FP64 FLOPs of the scatter kernel for one frame."""
    return (float(FP32_PER_SCAT_TEST * st["scat_tests"]),
            float(FP64_PER_CELL * st["scat_cells"] + FP64_PER_EVENT * st["scatter_events"]))


# Delay-and-sum (k_das), algorithmic work: per (pixel, transmit, element)
# term the sample index (1 add), the linear interpolation of a complex sample
# (2 x (2 mul + 1 add)) and its accumulation (2 adds); per (pixel, element)
# the receive distance (dx, dx^2 + dz^2, sqrt, scale: 5) and the apodised
# accumulation (complex fma: 4); per (pixel, transmit) the transmit delay
# (2 fma); per pixel the envelope (3 + sqrt).  Bytes: the channel data read
# once, IQ and envelope written once.
DAS_FLOP_PER_TERM = 9
DAS_FLOP_PER_PX_ELEM = 9
DAS_FLOP_PER_PX_TX = 4
DAS_FLOP_PER_PX = 4

TRACE_SOURCES = ["k_trace.hip", "k_bin.hip", "closest_hit.h", "trace_device.h", "scatter_grid.h", "scatter_grid.cpp", "bvh_layout.h", "philox.h", "ur_internal.h"]
DAS_SOURCES = ["k_signal.hip", "ur_internal.h"]


def kernel_hash(sources=TRACE_SOURCES):
    """Hash of a kernel's source (the .hip file, the headers it includes and
    its compile flags), to tell whether stored counter readings still apply."""
    from paper_2501_05828_amd import build as _build
    h = hashlib.sha256()
    h.update(" ".join(_build.EXTRA.get(sources[0], [])).encode())
    for name in sources:
        with open(os.path.join(ROOT, "paper_2501_05828_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_pmc(workload, kind="trace", sources=TRACE_SOURCES):
    """A committed rocprofv3 PMC summary (profiles/pmc_<kind>_<workload>.json),
    or None if absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kind}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash(sources):
        return None
    return d


def das_work(acq, grid):
    """Algorithmic FLOPs and bytes of one compounded DAS frame."""
    px = grid.nx * grid.nz
    T, E, S = acq.n_tx, acq.n_elements, acq.n_samples
    flops = px * (T * E * DAS_FLOP_PER_TERM + E * DAS_FLOP_PER_PX_ELEM + T * DAS_FLOP_PER_PX_TX + DAS_FLOP_PER_PX)
    nbytes = T * E * S * 8 + px * (8 + 4)
    return float(flops), float(nbytes), px * T * E


def das_roofline(workload, acq, grid, t_das):
    flops, nbytes, terms = das_work(acq, grid)
    out = {"kernel": "k_das", "bound": "alu", "achieved": flops / t_das / 1e12, "peak": PEAK_FP32 / 1e12,
           "unit": "TFLOP/s", "frac": flops / t_das / PEAK_FP32, "terms": terms,
           "hbm_achieved_gbs": nbytes / t_das / 1e9, "hbm_frac": nbytes / t_das / PEAK_HBM,
           "algorithmic_bytes": nbytes, "traffic": None, "valu": None}
    pmc = load_pmc(workload, "das", DAS_SOURCES)
    if pmc is not None:
        out["traffic"] = pmc["fetch_bytes"] / pmc["copy_fetch_factor"] + pmc["write_bytes"] / pmc["copy_write_factor"]
        v = pmc.get("valu")
        if v:
            out["valu"] = {"insts": v["insts"], "issue_frac": v["insts"] / (N_CU * CLOCK_HZ * t_das),
                           "lanes_active_frac": v["active_lanes_per_inst"] / 64.0}
    return out


def c3_measure(reps_trace=2, reps_das=10):
    """The batched workload (21 plane waves -20..20 deg, 2e7 rays per
    transmit, 1024 x 1024 Hann-apodised compound): trace rays/s and the DAS
    frame on its traced channel data, each from HIP events the library records
    around its kernels."""
    import torch

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.sim import Simulator

    w = scenes.batched()
    sim = Simulator(w)
    sim.trace(seed=w.seed + 7000)              # warm-up; leaves channel data for the DAS timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = []
    for i in range(reps_trace):
        sim.trace(seed=w.seed + 7001 + i)
        tr.append(sim.kernel_ms()[0])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps_trace
    sim.beamform()
    das = []
    for _ in range(reps_das):
        sim.beamform()
        das.append(sim.kernel_ms()[1])
    torch.cuda.synchronize()
    t_das = sum(das) / len(das) * 1e-3
    n_rays = w.acq.n_rays
    print(f"[bench] batched: trace {sum(tr) / len(tr):.1f} ms ({wall * 1e3:.1f} ms wall incl. secondary rays "
          f"and pulse), DAS {t_das * 1e3:.3f} ms", file=sys.stderr, flush=True)
    return {"workload": "batched: bone phantom, 128 elements, 21 plane waves -20..20 deg, "
                        f"{w.acq.n_elements * w.acq.rays_per_element:.2e} rays/transmit, DAS "
                        f"{w.grid.nx}x{w.grid.nz} Hann over 21x128x4096 channels",
            "rays_per_frame": n_rays, "trace_rays_per_s": n_rays / wall, "trace_frame_ms": wall * 1e3,
            "trace_kernel_ms": sum(tr) / len(tr), "das_kernel_ms": t_das * 1e3, "das_frames_per_s": 1.0 / t_das,
            "das_roofline": das_roofline("batched", w.acq, w.grid, t_das)}


def backward_measure(ray_stride=1):
    """The differentiable large scene (192 elements, 21 plane waves, two
    250k-triangle tubes, 4 spheres, 1e6 scatterers, linear binning) at full
    size: the forward trace and the path-replay adjoint of all gradient
    families at once (1e6 scatterer amplitudes, 6 attenuations, 6
    impedances, 12 sphere-centre coordinates) for a fixed random channel-data
    adjoint, each timed from the host around a synchronised call."""
    import numpy as np
    import torch

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.sim import Simulator

    w = scenes.large()
    sim = Simulator(w)
    A, sc = w.acq, w.scene
    rng = np.random.default_rng(41)
    g = torch.from_numpy(rng.normal(size=(A.n_tx, A.n_elements, A.n_samples)).astype(np.float32)).cuda()
    nm, ns, K = len(sc.materials), len(sc.sph), len(sc.scat)
    amp = torch.empty(K, device="cuda")
    al = torch.empty(nm, dtype=torch.float64, device="cuda")
    Z = torch.empty(nm, dtype=torch.float64, device="cuda")
    cen = torch.empty((ns, 3), dtype=torch.float64, device="cuda")

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    fwd = lambda: sim.trace(pulse=False, ray_stride=ray_stride)
    bwd = lambda: sim.ctx.ur_trace_adjoint(w.seed, g, amp=amp, alpha=al, Z=Z, sph_center=cen,
                                           ray_stride=ray_stride, frozen_choice=True)
    timed(fwd)
    t_f = timed(fwd)
    timed(bwd)
    t_b = timed(bwd)
    per_el = (A.rays_per_element + ray_stride - 1) // ray_stride
    paths = A.n_tx * A.n_elements * per_el
    print(f"[bench] backward: forward {t_f * 1e3:.1f} ms, adjoint {t_b * 1e3:.1f} ms ({t_b / t_f:.1f} x)",
          file=sys.stderr, flush=True)
    return {"workload": "differentiable large scene: 192 elements, 21 plane waves, two 250k-triangle tubes, "
                        "4 spheres, 1e6 scatterers, linear binning, every path of the frame",
            "paths": paths, "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3,
            "backward_paths_per_s": paths / t_b, "x_forward": t_b / t_f,
            "gradients": {"amplitudes": K, "attenuations": nm, "impedances": nm, "sphere_coordinates": 3 * ns},
            "directions_per_tangent_pass": 2}


def load_traffic(workload):
    """HBM bytes per launch of the extend kernel (the frame's total over its
    launches, divided by their number) from the committed rocprofv3 PMC
    summary, or None."""
    d = load_pmc(workload)
    if d is None:
        return None
    per_frame = d["fetch_bytes"] / d["copy_fetch_factor"] + d["write_bytes"] / d["copy_write_factor"]
    return per_frame / d["launches_per_frame"]


def cpu_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(workload, target_rays):
    from oracle import oracle as O
    nel = workload.acq.rays_per_element
    per_el = max(1, target_rays // (workload.acq.n_tx * workload.acq.n_elements))
    stride = max(1, nel // per_el)
    threads = cpu_threads()
    t0 = time.perf_counter()
    _, st = O.trace(workload, n_threads=threads, ray_stride=stride)
    dt = time.perf_counter() - t0
    return {"value": st["rays"] / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th ray of each (transmit, element): {st['rays']} rays of the same "
                      f"workload traced in {dt:.1f} s (FP64, brute-force intersection)"}


def learned_experiment(args):
    """Channel-data MSE against GPU time for uniform and learned emission on
    the bone phantom: reference = mean of uniform traces totalling 1e9 rays per
    transmit; MSE of Re(ch_rf) over the samples at round-trip depths of at
    least --min-depth-mm; time = device time of trace (including the
    secondary-ray kernel) and pulse shaping, proposal inference included."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.proposal import Proposal
    from paper_2501_05828_amd.sim import Simulator

    # the bone phantom (linear array), or the paper's acquisition settings on
    # the convex array with --workload convex
    w = scenes.convex() if args.workload == "convex" else scenes.learned()
    if args.element_choice == "cone":
        w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, element_choice=scenes.ELEMENT_CONE))
    acq0 = w.acq
    E, T = acq0.n_elements, acq0.n_tx
    sim = Simulator(w)

    def set_rays(per_tx):
        sim.set_acquisition(dataclasses.replace(acq0, rays_per_element=max(1, int(per_tx) // E)))

    def timed_trace(seed):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sim.trace(seed=seed, pulse=True)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) * 1e-3

    t0 = time.perf_counter()
    set_rays(args.ref_rays_per_tx / args.ref_parts)
    # the near field (scatterers within millimetres of the face, where the
    # 1/r^2 of transducer sampling makes the estimator heavy-tailed) is left
    # out of the MSE: samples of round-trip depth >= min_depth only
    n0 = int(np.ceil(2.0 * args.min_depth_mm * 1e-3 / acq0.c0 * acq0.f_s))
    ref = torch.zeros_like(sim.ch_rf[..., n0:, 0], dtype=torch.float64)
    for k in range(args.ref_parts):
        timed_trace(0xAB000000 + k)
        ref += sim.ch_rf[..., n0:, 0].double()
    ref /= args.ref_parts
    t_ref = time.perf_counter() - t0
    print(f"[learned] reference {args.ref_rays_per_tx:.1e} rays/tx in {t_ref:.1f} s", file=sys.stderr, flush=True)

    prop = Proposal(sim)
    set_rays(1e7)
    t0 = time.perf_counter()
    n_rec, offered = prop.record(args.record_traces, cap=args.record_cap, cost_aware=args.target == "cost")
    if offered > n_rec:
        # the buffer keeps the first records written (the first launch
        # ranges): later transmits would go untrained
        print(f"[learned] warning: {offered} records offered, {n_rec} kept; raise --record-cap",
              file=sys.stderr, flush=True)
    losses = prop.train(steps=args.train_steps, batch=1 << 16, lr=1e-3, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"[learned] {n_rec} records, {args.train_steps} steps in {t_train:.1f} s, loss {losses}",
          file=sys.stderr, flush=True)

    budgets = [float(b) for b in args.budgets.split(",")]
    curves = {"uniform": [], "learned": []}
    for mode in ("uniform", "learned"):
        for bi, per_tx in enumerate(budgets):
            set_rays(per_tx)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            if mode == "learned":
                prop.enable(args.epsilon)
            else:
                prop.disable()
            b.record()
            b.synchronize()
            t_inf = a.elapsed_time(b) * 1e-3 if mode == "learned" else 0.0
            reps = args.reps
            mse, tg = 0.0, 0.0
            for r in range(reps):
                tg += timed_trace(0xCD000000 + 97 * bi + r + (0 if mode == "uniform" else 50000))
                mse += float(((sim.ch_rf[..., n0:, 0].double() - ref) ** 2).mean())
            curves[mode].append({"rays_per_tx": per_tx, "mse": mse / reps, "gpu_s": tg / reps + t_inf})
            print(f"[learned] {mode} {per_tx:.0e}/tx: mse {mse / reps:.4e} time {tg / reps + t_inf:.4f} s",
                  file=sys.stderr, flush=True)
    # time uniform needs to reach each learned MSE (log-log interpolation)
    lu = np.log([c["mse"] for c in curves["uniform"]])
    tu = np.log([c["gpu_s"] for c in curves["uniform"]])
    ratios = []
    for c in curves["learned"]:
        m = np.log(c["mse"])
        if lu.min() <= m <= lu.max():
            order = np.argsort(lu)
            t_u = float(np.exp(np.interp(m, lu[order], tu[order])))
            ratios.append({"rays_per_tx": c["rays_per_tx"], "learned_s": c["gpu_s"], "uniform_s_same_mse": t_u,
                           "time_ratio": c["gpu_s"] / t_u})
    # efficiency = 1 / (MSE x time): its ratio is the speed-up of the
    # learned proposal at equal MSE while both are variance-dominated
    gains = [{"rays_per_tx": u["rays_per_tx"],
              "efficiency_gain": (u["mse"] * u["gpu_s"]) / (l["mse"] * l["gpu_s"])}
             for u, l in zip(curves["uniform"], curves["learned"])]
    wl_name = "convex array, the paper's acquisition settings" if args.workload == "convex" else "bone phantom (learned)"
    out = {"metric": "channel MSE at equal GPU time, learned vs uniform", "workload": wl_name,
           "target": args.target, "element_choice": args.element_choice, "epsilon": args.epsilon, "reps": args.reps,
           "min_depth_mm": args.min_depth_mm, "efficiency_gain": gains,
           "reference_rays_per_tx": args.ref_rays_per_tx, "records": n_rec, "records_offered": offered,
           "train_steps": args.train_steps, "train_s": t_train, "loss_log": losses, "curves": curves,
           "learned_time_over_uniform_time_at_equal_mse": ratios}
    print(json.dumps(out))


def rough_nee_experiment(args):
    """Channel-data MSE against GPU time on the bone phantom with the bone's
    roughness 0.5, with and without transducer sampling at the rough
    boundaries (direct hits only): one reference per arm (mean of traces of
    that arm, --ref-rays-per-tx in total), whose difference in total signal
    is reported with its standard error; MSE of Re(ch_rf) beyond
    --min-depth-mm against the arm's own reference; time = device time of
    trace + pulse."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.sim import Simulator

    w = scenes.bone_rough()
    if args.element_choice == "cone":
        w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, element_choice=scenes.ELEMENT_CONE))
    acq0 = w.acq
    E = acq0.n_elements
    sim = Simulator(w)

    def run(per_tx, direct_only, seed):
        sim.set_acquisition(dataclasses.replace(acq0, rays_per_element=max(1, int(per_tx) // E),
                                                rough_direct_only=direct_only))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sim.trace(seed=seed, pulse=True)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) * 1e-3

    n0 = int(np.ceil(2.0 * args.min_depth_mm * 1e-3 / acq0.c0 * acq0.f_s))
    # one reference per arm: their difference (with its standard error from
    # the spread of the parts) tests that both estimate the same data
    refs, totals = {}, {}
    for direct_only in (0, 1):
        ref = torch.zeros_like(sim.ch_rf[..., n0:, 0], dtype=torch.float64)
        tot = []
        for k in range(args.ref_parts):
            run(args.ref_rays_per_tx / args.ref_parts, direct_only, 0xAB000000 + k + 1000 * direct_only)
            ref += sim.ch_rf[..., n0:, 0].double()
            tot.append(float(sim.ch_raw.double().sum()))
        refs[direct_only] = ref / args.ref_parts
        totals[direct_only] = np.array(tot)
    ref = refs[0]
    t0, t1 = totals[0], totals[1]
    bias = {"total_signal_with_rough_sampling": float(t0.mean()), "total_signal_direct_only": float(t1.mean()),
            "difference": float(t0.mean() - t1.mean()),
            "difference_se": float(np.sqrt(t0.var(ddof=1) / len(t0) + t1.var(ddof=1) / len(t1))),
            "reference_mse_between_arms": float(((refs[0] - refs[1]) ** 2).mean())}
    print(f"[rough-nee] references: {json.dumps(bias)}", file=sys.stderr, flush=True)
    curves = {"direct_only": [], "with_rough_sampling": []}
    for mode, direct_only in (("direct_only", 1), ("with_rough_sampling", 0)):
        for bi, per_tx in enumerate(float(b) for b in args.budgets.split(",")):
            mse, tg = 0.0, 0.0
            for r in range(args.reps):
                tg += run(per_tx, direct_only, 0xCD000000 + 97 * bi + r + 50000 * direct_only)
                mse += float(((sim.ch_rf[..., n0:, 0].double() - refs[direct_only]) ** 2).mean())
            curves[mode].append({"rays_per_tx": per_tx, "mse": mse / args.reps, "gpu_s": tg / args.reps})
            print(f"[rough-nee] {mode} {per_tx:.0e}/tx: mse {mse / args.reps:.4e} time {tg / args.reps:.4f} s",
                  file=sys.stderr, flush=True)
    gains = [{"rays_per_tx": a["rays_per_tx"], "efficiency_gain": (a["mse"] * a["gpu_s"]) / (b["mse"] * b["gpu_s"])}
             for a, b in zip(curves["direct_only"], curves["with_rough_sampling"])]
    print(json.dumps({"metric": "channel MSE at equal GPU time, rough-boundary transducer sampling vs direct hits only",
                      "workload": "bone phantom, bone roughness 0.5", "element_choice": args.element_choice,
                      "reps": args.reps, "min_depth_mm": args.min_depth_mm,
                      "reference_rays_per_tx": args.ref_rays_per_tx, "references": bias, "efficiency_gain": gains,
                      "curves": curves}))


def edges_experiment(args):
    """The direct-hit edge terms (ur_trace_grad_edges) against common-random-
    number differences of the expected data.  The small scene with its
    sphere under the aperture (12 mm deep, radius 3 mm), no scatterers,
    linear binning, receive angles 10 / 45 degrees, args.edge_rays rays per
    element, a linear array or (args.edge_convex) a convex one of 20 mm
    radius, without scatterers or (args.edge_scatterers) with the scene's
    2000; the channel adjoint g is one smooth random time profile (white
    noise filtered by a Gaussian of 40 samples) with one sign per half of the
    aperture, so it jumps at the centre edge, or (args.edge_adjoint random)
    such noise drawn for every element.  For every key (Philox seed):
    J(x_c +- h) of the sphere centre's x from the replay's FP64 functional,
    the interior adjoint (choice attached) and the edge terms.  Prints one
    JSON line with the means and standard errors over the keys."""
    import dataclasses
    import math

    import numpy as np
    import torch
    from scipy.ndimage import gaussian_filter1d

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.sim import Simulator

    w = scenes.tiny(rays_per_element=args.edge_rays)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45), binning=scenes.LINEAR,
                              angles=np.deg2rad([0.0]))
    sph = np.array([[1.0e-3, 0.5e-3, 12.0e-3, 3.0e-3]])
    scat = w.scene.scat if args.edge_scatterers else np.zeros((0, 4))
    sc = dataclasses.replace(w.scene, sph=sph, sph_mat=np.array([[0, 2]], np.int32), scat=scat)
    w = dataclasses.replace(w, acq=acq, scene=sc)
    if args.edge_convex:
        w = scenes.convex_probe(w, 20e-3)
    A = w.acq
    rng = np.random.default_rng(5)
    if args.edge_adjoint == "step":
        prof = np.abs(gaussian_filter1d(rng.normal(size=A.n_samples), 40.0) * 10)
        sign = np.where(np.arange(A.n_elements) < A.n_elements // 2, 1.0, -1.0)
        gn = prof[None, None, :] * sign[None, :, None]
    else:
        gn = gaussian_filter1d(rng.normal(size=(A.n_tx, A.n_elements, A.n_samples)), 40.0, axis=2) * 10
    g = torch.from_numpy(gn.astype(np.float32)).cuda()
    sim = Simulator(w)
    ctx = sim.ctx
    hs = (1e-4, 1e-5, 2e-6)
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    cen = torch.empty((1, 3), dtype=torch.float64, device="cuda")

    def J(seed, dx):
        s2 = sph.copy()
        s2[0, 0] += dx
        ctx.ur_scene_update(sph=s2)
        ctx.ur_trace_adjoint(seed, g, value=v)
        return float(v.item())

    fd = {h: [] for h in hs}
    interior, edges = [], []
    t0 = time.perf_counter()
    for key in range(args.edge_keys):
        seed = w.seed + 1000 * key
        for h in hs:
            fd[h].append((J(seed, h) - J(seed, -h)) / (2 * h))
        ctx.ur_scene_update(sph=sph)
        ctx.ur_trace_adjoint(seed, g, sph_center=cen, frozen_choice=False)
        interior.append(float(cen[0, 0].item()))
        ctx.ur_trace_grad_edges(seed, g, sph_center=cen)
        edges.append(float(cen[0, 0].item()))
        if (key + 1) % 500 == 0:
            print(f"[edges] {key + 1} keys, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)

    def stat(x):
        x = np.asarray(x)
        return {"mean": float(x.mean()), "se": float(x.std(ddof=1) / math.sqrt(len(x)))}

    it, ed = np.asarray(interior), np.asarray(edges)
    array = "convex array of 20 mm radius" if args.edge_convex else "linear array"
    scat_note = f"{len(w.scene.scat)} scatterers" if args.edge_scatterers else "no scatterers"
    out = {"experiment": "edge_terms", "workload": f"small scene, sphere under the aperture, {scat_note}, "
           f"{array}, {A.n_elements} elements x {A.rays_per_element} rays, adjoint "
           + ("with one sign per half aperture" if args.edge_adjoint == "step" else "random per element"),
           "keys": args.edge_keys, "parameter": "sphere centre x",
           "differences": {f"h={h:g} m": stat(fd[h]) for h in hs},
           "interior": stat(it), "edge_terms": stat(ed), "interior_plus_edges": stat(it + ed),
           "seconds": time.perf_counter() - t0}
    print(json.dumps(out))


def binning_experiment(args):
    """Records per frame and trace time of the bone frame under four receive
    configurations: the uniform and the cone-restricted element choice at the
    2-degree cone, the cone choice with a trained proposal, and a 45-degree
    receive cone (alpha_m 15 degrees) with either choice.  Each record is one
    float atomic into the channel data (two with linear binning)."""
    import dataclasses
    import math

    import torch

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.proposal import Proposal
    from paper_2501_05828_amd.sim import Simulator

    w0 = scenes.bone()
    base = w0.acq
    wide = dict(alpha_m=math.radians(15), alpha_c=math.radians(45))
    cfgs = [("uniform", base), ("cone", dataclasses.replace(base, element_choice=scenes.ELEMENT_CONE)),
            ("cone_learned", dataclasses.replace(base, element_choice=scenes.ELEMENT_CONE)),
            ("uniform_45deg", dataclasses.replace(base, **wide)),
            ("cone_45deg", dataclasses.replace(base, element_choice=scenes.ELEMENT_CONE, **wide))]
    sim = Simulator(w0)

    def timed(seed):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sim.trace(seed=seed, pulse=False)
        b.record()
        b.synchronize()
        return a.elapsed_time(b)

    out = {}
    for name, acq in cfgs:
        sim.set_acquisition(acq)
        prop = None
        if name == "cone_learned":
            prop = Proposal(sim)
            prop.record(8, cap=1 << 26, cost_aware=True)
            prop.train(steps=2000)
            prop.enable(0.1)
        st = sim.trace(seed=5, stats=True, pulse=False)
        timed(6)
        ts = [timed(7 + i) for i in range(5)]
        xm, sm, nm, _ = sim.ctx.ur_last_trace_kernels_ms()
        out[name] = {"records_per_frame": st["records"], "trace_ms": sum(ts) / len(ts), "extend_ms": xm,
                     "scatter_ms": sm, "secondary_ray_ms": nm}
        if prop is not None:
            prop.disable()
        print(f"[binning] {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)
    print(json.dumps({"experiment": "binning", "workload": "bone", "configs": out}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bone", choices=["bone", "batched", "tiny", "convex", "bone_rough", "paper"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=150000)
    ap.add_argument("--experiment", choices=["learned", "rough-nee", "binning", "edges"], default=None,
                    help="learned: channel MSE vs GPU time, learned vs uniform emission; rough-nee: with vs "
                         "without transducer sampling at the rough bone; binning: records per frame and trace time "
                         "under four receive configurations")
    ap.add_argument("--ref-rays-per-tx", type=float, default=1e9)
    ap.add_argument("--ref-parts", type=int, default=10)
    ap.add_argument("--record-traces", type=int, default=8)
    ap.add_argument("--record-cap", type=int, default=1 << 27, help="contribution records kept (8 B each)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--target", choices=["abs", "cost"], default="cost",
                    help="proposal target per cell: sum |c|, or sqrt(sum c^2 / path cost)")
    ap.add_argument("--reps", type=int, default=3, help="independent traces per budget (MSE averaged)")
    ap.add_argument("--epsilon", type=float, default=0.1, help="uniform share of the learned emission mixture")
    ap.add_argument("--min-depth-mm", type=float, default=5.0, help="MSE over samples at this round-trip depth and beyond")
    ap.add_argument("--budgets", default="1e6,3e6,1e7,3e7", help="rays per transmit, comma-separated")
    ap.add_argument("--element-choice", choices=["uniform", "cone"], default="uniform",
                    help="transducer-sampling target: uniform over all elements, or over those in the cone")
    ap.add_argument("--print-kernel-hash", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched-workload trace and DAS measurement")
    ap.add_argument("--c3-only", action="store_true", help="run only the batched-workload trace and DAS measurement")
    ap.add_argument("--no-backward", action="store_true", help="skip the adjoint measurement on the large scene")
    ap.add_argument("--edge-keys", type=int, default=4000, help="keys of --experiment edges")
    ap.add_argument("--edge-rays", type=int, default=2048, help="rays per element of --experiment edges")
    ap.add_argument("--edge-convex", action="store_true", help="--experiment edges through a 20 mm convex array")
    ap.add_argument("--edge-adjoint", choices=["step", "random"], default="step",
                    help="--experiment edges: one time profile signed per half aperture, or smooth random per element")
    ap.add_argument("--edge-scatterers", action="store_true",
                    help="--experiment edges with the small scene's 2000 scatterers (their capture terms are not built)")
    ap.add_argument("--backward-only", action="store_true", help="run only the adjoint measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(json.dumps({"trace": kernel_hash(), "das": kernel_hash(DAS_SOURCES)}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (rays would shard by transmit "
              "and element rows, with one reduction of the channel data)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.experiment == "learned":
        learned_experiment(args)
        return
    if args.experiment == "rough-nee":
        rough_nee_experiment(args)
        return
    if args.experiment == "binning":
        binning_experiment(args)
        return
    if args.experiment == "edges":
        edges_experiment(args)
        return
    if args.backward_only:
        print(json.dumps(backward_measure()))
        return
    if args.c3_only:
        print(json.dumps(c3_measure()))
        return
    if args.copy_calibration:
        a = torch.ones(1 << 28, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "launches": 3}))
        return

    from paper_2501_05828_amd import scenes
    from paper_2501_05828_amd.sim import Simulator

    w = scenes.make(args.workload)
    sim = Simulator(w)
    acq, grid = w.acq, w.grid
    n_rays = acq.n_rays
    print(f"[bench] {w.name}: {n_rays:.3e} rays/frame, grid {grid.nx}x{grid.nz}", file=sys.stderr, flush=True)

    # instrumented pass: unit counts for the algorithmic FLOPs of one frame
    st = sim.trace(seed=w.seed, stats=True)
    xf32, xf64 = extend_flops(st, len(w.scene.pln), len(w.scene.sph))
    sf32, sf64 = scatter_flops(st)
    print(f"[bench] counting pass: {st['kernel_ms']:.1f} ms, records {st['records']}", file=sys.stderr, flush=True)
    print(f"[bench] counts {json.dumps(st)}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        sim.step(seed=w.seed + 1000 + i)
    torch.cuda.synchronize()
    trace_ms, das_ms, ext_ms, sca_ms = [], [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        sim.step(seed=w.seed + i)
        tm, dm = sim.kernel_ms()
        xm, sm, _, launches = sim.ctx.ur_last_trace_kernels_ms()
        trace_ms.append(tm)
        das_ms.append(dm)
        ext_ms.append(xm)
        sca_ms.append(sm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    mean = lambda v: sum(v) / len(v) * 1e-3
    t_trace, t_das, t_ext, t_sca = mean(trace_ms), mean(das_ms), mean(ext_ms), mean(sca_ms)
    print(f"[bench] {ms_step:.1f} ms/step, trace {1e3 * t_trace:.1f} ms (extend {1e3 * t_ext:.1f}, "
          f"scatter {1e3 * t_sca:.1f}), DAS {1e3 * t_das:.3f} ms", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (extend): FLOPs of one frame over its
    # launch time summed over the frame's launches
    achieved = (xf32 + xf64) / t_ext
    peak = (xf32 + xf64) / (xf32 / PEAK_FP32 + xf64 / PEAK_FP64)
    traffic = load_traffic(w.name)
    pmc = load_pmc(w.name)
    das_roof = das_roofline(w.name, acq, grid, t_das)
    valu = None
    if pmc is not None and "valu" in pmc:
        # a wave64 VALU instruction occupies one 16-lane SIMD for 4 cycles:
        # 4 SIMDs per CU issue at most one wave instruction per CU per cycle
        insts = pmc["valu"]["insts_per_frame"]
        valu = {"insts_per_frame": insts,
                "issue_frac": insts / (N_CU * CLOCK_HZ * t_ext),
                "lanes_active_frac": pmc["valu"]["active_lanes_per_inst"] / 64.0}
    out = {
        "metric": METRIC,
        "value": n_rays * args.steps / elapsed,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 decisions, f32 data",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name} phantom: {acq.n_elements} elements"
                        + (f" on a {acq.radius * 1e3:.0f} mm convex arc" if acq.radius > 0 else "")
                        + f", {acq.n_tx} plane waves "
                        f"{round(float(acq.angles[0]) * 57.29578)}..{round(float(acq.angles[-1]) * 57.29578)} deg, "
                        f"{acq.n_elements * acq.rays_per_element:.2e} rays/transmit, {acq.max_bounces} bounces, "
                        f"{len(w.scene.tri)} triangles, {len(w.scene.pln)} planes, {len(w.scene.sph)} spheres, "
                        f"{len(w.scene.scat)} scatterers, "
                        + (f"GGX roughness {max(w.scene.rough):g} on the bone, " if w.scene.rough is not None
                           and max(w.scene.rough) > 0 else "")
                        + f"{acq.n_samples} samples at {acq.f_s / 1e6:.0f} MHz, "
                        + (f"DAS on a {grid.nx}x{grid.nz} sector grid, scan converted to "
                         f"{w.extra['cart_grid'].nx}x{w.extra['cart_grid'].nz}" if grid.sector
                         else f"DAS {grid.nx}x{grid.nz}"),
            "rays_per_frame": n_rays,
            "scene_seed": w.scene_seed,
        },
        "frames_per_s": args.steps / elapsed,
        "das_frames_per_s": 1.0 / t_das,
        "trace_kernel_ms": 1e3 * t_trace,
        "extend_kernel_ms": 1e3 * t_ext,
        "scatter_kernel_ms": 1e3 * t_sca,
        "das_kernel_ms": 1e3 * t_das,
        "roofline": {
            "kernel": "k_extend",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "flops_fp32": xf32,
            "flops_fp64": xf64,
            "launches_per_frame": launches,
            "kernel_ms_per_launch": 1e3 * t_ext / launches,
            "valu": valu,
        },
        "scatter_kernel": {
            "ms": 1e3 * t_sca,
            "achieved_tflops": (sf32 + sf64) / t_sca / 1e12 if t_sca > 0 else None,
            "flops_fp32": sf32,
            "flops_fp64": sf64,
        },
        "das_roofline": das_roof,
    }
    if not args.no_c3 and w.name == "bone":
        out["batched"] = c3_measure()
    if not args.no_backward and w.name == "bone":
        out["backward"] = backward_measure()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_rays)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
