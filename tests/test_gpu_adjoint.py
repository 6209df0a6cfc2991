"""GPU adjoint: transposed signal chain and path-replay trace gradients.

Linear operators (pulse convolution, delay-and-sum) are checked by the
adjoint identity <A x, y> = <x, A^T y> on seeded random data.  The trace
gradients are checked against central finite differences of the FP64
oracle's channel data for the same seed, J(p) = sum g * ch_raw(p):

* amplitudes: J is linear in them, so the difference quotient is exact;
* attenuation: J is smooth and no decision depends on it;
* impedance and sphere centres: with the reflect-or-transmit choice frozen,
  J is smooth between decision changes; a step is accepted only if every
  integer trace counter is the same at p - h, p and p + h (no decision
  changed), otherwise the step is reduced.

The attached choice probability (the default) adds a score term whose mean
is the derivative of the expected data; it is checked statistically against
common-random-number differences of the GPU forward over many seeds in a
scene where only that term is non-zero.

Every gradient is also compared element by element with the oracle's FP64
forward-mode gradient of the same paths (or_trace_grad, pinned on the CPU
against finite differences of the oracle's forward trace): the small scene
(frozen and attached choice), a convex array, the bone phantom, and the
differentiable large scene at full size on a stride sample.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

pytestmark = pytest.mark.gpu

EXACT_STATS = ["rays", "segments", "reflect", "transmit", "tir", "scatter_events", "nee_zero", "nee_cast",
               "nee_blocked", "direct_hits", "records", "dropped", "term_box", "term_bounce", "term_time",
               "term_path"]


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _workload(rays=1024, binning=scenes.LINEAR, angles_deg=(0.0,)):
    """Small scene with its sphere moved under the aperture (centre 12 mm
    deep), so that paths meet it."""
    w = scenes.tiny(rays_per_element=rays)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45), binning=binning,
                              angles=np.deg2rad(np.asarray(angles_deg, np.float64)))
    sph = np.array([[1.0e-3, 0.5e-3, 12.0e-3, 3.0e-3]])
    return dataclasses.replace(w, acq=acq, scene=dataclasses.replace(w.scene, sph=sph,
                                                                     sph_mat=np.array([[0, 2]], np.int32)))


def _with_scene(w, **kw):
    return dataclasses.replace(w, scene=dataclasses.replace(w.scene, **kw))


def _smooth_adjoint(shape, seed, sigma=8.0):
    """Seeded adjoint of the channel data: white noise smoothed along time by a
    Gaussian of `sigma` samples (slopes change little from sample to sample)."""
    rng = np.random.default_rng(seed)
    x = rng.normal(size=shape)
    k = np.arange(-int(4 * sigma), int(4 * sigma) + 1)
    ker = np.exp(-0.5 * (k / sigma) ** 2)
    ker /= np.sqrt((ker ** 2).sum())
    y = np.apply_along_axis(lambda r: np.convolve(r, ker, mode="same"), -1, x)
    return y.astype(np.float32)


def _J(oracle, w, g):
    """J, the integer trace counters and the set of non-empty bins (a path
    that moves to another element or time bin changes the set)."""
    ch, st = oracle.trace(w)
    key = ({k: st[k] for k in EXACT_STATS}, np.flatnonzero(ch).tobytes())
    return float(np.sum(g.astype(np.float64) * ch)), key


def _fd(oracle, w, g, perturb, h0, tries=4):
    """Central difference of J along `perturb(w, h)`, reducing h until no
    decision differs between the three points; None if none is clean."""
    _, k0 = _J(oracle, w, g)
    h = h0
    for _ in range(tries):
        jp, kp = _J(oracle, perturb(w, h), g)
        jm, km = _J(oracle, perturb(w, -h), g)
        if kp == k0 and km == k0:
            return (jp - jm) / (2 * h), h
        h *= 0.1
    return None, h


def _sim(w):
    from paper_2501_05828_amd.sim import Simulator
    return Simulator(w)


# ------------------------------------------------------------ linear operators
def test_pulse_adjoint_identity(torch_gpu):
    torch = torch_gpu
    w = _workload(rays=1, angles_deg=(-5.0, 0.0, 5.0))
    s = _sim(w)
    gen = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn(s.ch_raw.shape, device="cuda", generator=gen)
    y = torch.randn(s.ch_rf.shape, device="cuda", generator=gen)
    ax = torch.empty_like(s.ch_rf)
    s.ctx.ur_pulse(x, ax)
    aty = torch.empty_like(s.ch_raw)
    s.ctx.ur_pulse_adjoint(y, aty)
    lhs = float((ax.double() * y.double()).sum())
    rhs = float((x.double() * aty.double()).sum())
    print(f"[adjoint] pulse <Ax,y>={lhs:.9e} <x,ATy>={rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * float(ax.double().norm() * y.double().norm())


@pytest.mark.parametrize("apod", ["hann", "none"])
def test_das_adjoint_identity(torch_gpu, apod):
    torch = torch_gpu
    from paper_2501_05828_amd import binding
    w = _workload(rays=1, angles_deg=(-5.0, 0.0, 5.0))
    w = dataclasses.replace(w, apod=apod)
    s = _sim(w)
    ap = binding.UR_APOD_HANN if apod == "hann" else binding.UR_APOD_NONE
    gen = torch.Generator(device="cuda").manual_seed(12)
    rf = torch.randn(s.ch_rf.shape, device="cuda", generator=gen)
    y = torch.randn(s.iq.shape, device="cuda", generator=gen)
    iq = torch.empty_like(s.iq)
    s.ctx.ur_beamform(w.grid, rf, iq=iq, apod=ap)
    g_rf = torch.empty_like(s.ch_rf)
    s.ctx.ur_beamform_adjoint(w.grid, g_rf, g_iq=y, apod=ap)
    lhs = float((iq.double() * y.double()).sum())
    rhs = float((rf.double() * g_rf.double()).sum())
    print(f"[adjoint] das/{apod} <Ax,y>={lhs:.9e} <x,ATy>={rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * float(iq.double().norm() * y.double().norm())
    # samples never read by the beamformer receive no gradient
    assert float(g_rf.abs().sum()) > 0


def test_envelope_adjoint_matches_autograd(torch_gpu):
    """The envelope path of ur_beamform_adjoint equals the IQ path fed with
    the derivative of |IQ| that torch's autograd gives."""
    torch = torch_gpu
    w = _workload(rays=1)
    s = _sim(w)
    gen = torch.Generator(device="cuda").manual_seed(13)
    rf = torch.randn(s.ch_rf.shape, device="cuda", generator=gen)
    iq = torch.empty_like(s.iq)
    s.ctx.ur_beamform(w.grid, rf, iq=iq)
    g_env = torch.randn(s.env.shape, device="cuda", generator=gen)
    z = iq.double().clone().requires_grad_(True)
    env = torch.sqrt((z * z).sum(-1))
    (env * g_env.double()).sum().backward()
    g_iq = z.grad.float().contiguous()
    a = torch.empty_like(s.ch_rf)
    b = torch.empty_like(s.ch_rf)
    s.ctx.ur_beamform_adjoint(w.grid, a, iq=iq, g_env=g_env)
    s.ctx.ur_beamform_adjoint(w.grid, b, g_iq=g_iq)
    err = float((a.double() - b.double()).norm() / b.double().norm())
    print(f"[adjoint] envelope rel_l2={err:.2e}", flush=True)
    assert err <= 1e-4


# ------------------------------------------------------------ trace adjoint
@pytest.fixture(scope="module")
def tiny_adj(torch_gpu):
    torch = torch_gpu
    w = _workload()
    g = _smooth_adjoint((w.acq.n_tx, w.acq.n_elements, w.acq.n_samples), 21)
    s = _sim(w)
    return torch, w, g, s, torch.from_numpy(g).cuda()


def test_trace_adjoint_amplitudes(oracle, tiny_adj):
    torch, w, g, s, gt = tiny_adj
    K = len(w.scene.scat)
    amp = torch.empty(K, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, amp=amp)
    ga = amp.double().cpu().numpy()
    assert np.count_nonzero(ga) > 20
    rng = np.random.default_rng(5)
    a0 = w.scene.scat[:, 3].copy()

    def perturb(v):
        return lambda ww, h: _with_scene(ww, scat=np.column_stack([ww.scene.scat[:, :3], a0 + h * v]))

    dirs = [rng.normal(size=K) for _ in range(2)]
    top = np.argsort(-np.abs(ga))[:3]
    for k in top:
        e = np.zeros(K)
        e[k] = 1.0
        dirs.append(e)
    for v in dirs:
        fd, h = _fd(oracle, w, g, perturb(v), 1.0, tries=1)
        got = float(ga @ v)
        print(f"[adjoint] amp dir: gpu={got:.9e} fd={fd:.9e}", flush=True)
        assert fd is not None
        assert abs(got - fd) <= 1e-5 * np.linalg.norm(ga) * np.linalg.norm(v) + 1e-6 * abs(fd)


def test_trace_adjoint_attenuation(oracle, tiny_adj):
    torch, w, g, s, gt = tiny_adj
    nm = len(w.scene.materials)
    al = torch.empty(nm, dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, alpha=al)
    ga = al.cpu().numpy()
    for m in range(nm):
        def perturb(ww, h, m=m):
            mat = ww.scene.materials.copy()
            mat[m, 1] += h
            return _with_scene(ww, materials=mat)
        fd, h = _fd(oracle, w, g, perturb, 1e-4)
        print(f"[adjoint] dJ/dalpha[{m}]: gpu={ga[m]:.9e} fd={fd:.9e} (h={h:g})", flush=True)
        assert fd is not None
        assert abs(ga[m] - fd) <= 1e-5 * np.max(np.abs(ga)) + 1e-6 * abs(fd)


def test_trace_adjoint_impedance_and_sphere(oracle, tiny_adj):
    torch, w, g, s, gt = tiny_adj
    nm = len(w.scene.materials)
    Z = torch.empty(nm, dtype=torch.float64, device="cuda")
    sc = torch.empty((len(w.scene.sph), 3), dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, Z=Z, sph_center=sc, frozen_choice=True)
    gz, gs = Z.cpu().numpy(), sc.cpu().numpy().ravel()
    checked = 0
    for m in range(nm):
        def perturb(ww, h, m=m):
            mat = ww.scene.materials.copy()
            mat[m, 0] += h
            return _with_scene(ww, materials=mat)
        fd, h = _fd(oracle, w, g, perturb, 1e-6)
        print(f"[adjoint] dJ/dZ[{m}]: gpu={gz[m]:.9e} fd={fd} (h={h:g})", flush=True)
        if fd is None:
            continue
        checked += 1
        assert abs(gz[m] - fd) <= 1e-4 * max(np.max(np.abs(gz)), abs(fd))
    for c in range(gs.size):
        def perturb(ww, h, c=c):
            sph = ww.scene.sph.copy()
            sph[c // 3, c % 3] += h
            return _with_scene(ww, sph=sph)
        fd, h = _fd(oracle, w, g, perturb, 1e-9)
        print(f"[adjoint] dJ/dcentre[{c}]: gpu={gs[c]:.9e} fd={fd} (h={h:g})", flush=True)
        if fd is None:
            continue
        checked += 1
        assert abs(gs[c] - fd) <= 1e-4 * max(np.max(np.abs(gs)), abs(fd))
    assert checked >= nm + 1


def test_trace_adjoint_convex_array(oracle, torch_gpu):
    """The adjoint on a convex array (the array's cylinder as the exit face,
    element normals in the receive angle): attenuation, impedance and
    sphere-centre gradients against central differences of the oracle."""
    torch = torch_gpu
    w = scenes.convex_probe(_workload(), 20e-3)
    g = _smooth_adjoint((w.acq.n_tx, w.acq.n_elements, w.acq.n_samples), 22)
    s = _sim(w)
    gt = torch.from_numpy(g).cuda()
    nm = len(w.scene.materials)
    al = torch.empty(nm, dtype=torch.float64, device="cuda")
    Z = torch.empty(nm, dtype=torch.float64, device="cuda")
    sc = torch.empty((len(w.scene.sph), 3), dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, alpha=al, Z=Z, sph_center=sc, frozen_choice=True)
    ga, gz, gs = al.cpu().numpy(), Z.cpu().numpy(), sc.cpu().numpy().ravel()
    assert np.count_nonzero(ga) > 0
    checked = 0
    for m in range(nm):
        def perturb(ww, h, m=m):
            mat = ww.scene.materials.copy()
            mat[m, 1] += h
            return _with_scene(ww, materials=mat)
        fd, h = _fd(oracle, w, g, perturb, 1e-4)
        print(f"[adjoint] convex dJ/dalpha[{m}]: gpu={ga[m]:.9e} fd={fd} (h={h:g})", flush=True)
        assert fd is not None
        assert abs(ga[m] - fd) <= 1e-5 * np.max(np.abs(ga)) + 1e-6 * abs(fd)
    for m in range(nm):
        def perturb(ww, h, m=m):
            mat = ww.scene.materials.copy()
            mat[m, 0] += h
            return _with_scene(ww, materials=mat)
        fd, h = _fd(oracle, w, g, perturb, 1e-6)
        print(f"[adjoint] convex dJ/dZ[{m}]: gpu={gz[m]:.9e} fd={fd} (h={h:g})", flush=True)
        if fd is None:
            continue
        checked += 1
        assert abs(gz[m] - fd) <= 1e-4 * max(np.max(np.abs(gz)), abs(fd))
    for c in range(gs.size):
        def perturb(ww, h, c=c):
            sph = ww.scene.sph.copy()
            sph[c // 3, c % 3] += h
            return _with_scene(ww, sph=sph)
        fd, h = _fd(oracle, w, g, perturb, 1e-9)
        print(f"[adjoint] convex dJ/dcentre[{c}]: gpu={gs[c]:.9e} fd={fd} (h={h:g})", flush=True)
        if fd is None:
            continue
        checked += 1
        assert abs(gs[c] - fd) <= 1e-4 * max(np.max(np.abs(gs)), abs(fd))
    assert checked >= nm + 1


# ------------------------------------------------ against the FP64 oracle gradient
def _gpu_grads(s, w, gt, stride=1, frozen=True, record_paths=0):
    import torch
    sc = w.scene
    nm, ns, K = len(sc.materials), len(sc.sph), len(sc.scat)
    Z = torch.empty(nm, dtype=torch.float64, device="cuda")
    al = torch.empty(nm, dtype=torch.float64, device="cuda")
    cg = torch.empty((ns, 3), dtype=torch.float64, device="cuda") if ns else None
    ag = torch.empty(K, device="cuda") if K else None
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, amp=ag, alpha=al, Z=Z, sph_center=cg, value=v, frozen_choice=frozen,
                           ray_stride=stride, record_paths=record_paths)
    return dict(J=float(v.item()), z=Z.cpu().numpy(), alpha=al.cpu().numpy(),
                sph=cg.cpu().numpy() if ns else np.zeros((0, 3)),
                amp=ag.double().cpu().numpy() if K else np.zeros(0))


def _assert_matches_oracle(got, ref, label):
    """Element by element: the FP64 families (impedance, attenuation, sphere
    centre; accumulated in FP64 on both sides, in another order) within 1e-8
    of their largest oracle entry, the amplitude gradients (FP32 atomics on
    the GPU) within 1e-6; entries the oracle leaves exactly zero (no replayed
    path depends on them) are exactly zero on the GPU too."""
    print(f"[adjoint-oracle] {label}: J gpu {got['J']:.12e} oracle {ref['J']:.12e}", flush=True)
    assert abs(got["J"] - ref["J"]) <= 1e-9 * abs(ref["J"]) + 1e-300
    for key, tol in (("z", 1e-8), ("alpha", 1e-8), ("sph", 1e-8), ("amp", 1e-6)):
        a, b = np.asarray(got[key]).ravel(), np.asarray(ref[key]).ravel()
        assert a.shape == b.shape
        if b.size == 0:
            continue
        scale = np.abs(b).max()
        err = np.abs(a - b).max()
        print(f"[adjoint-oracle] {label}: {key} max|oracle| {scale:.4e} max err {err:.3e} "
              f"nonzero {np.count_nonzero(b)}/{b.size}", flush=True)
        assert np.array_equal(a[b == 0], b[b == 0]), key
        assert err <= tol * scale, (key, err, scale)


@pytest.mark.parametrize("frozen", [True, False])
def test_trace_adjoint_matches_oracle_gradient(oracle, tiny_adj, frozen):
    """Every gradient of the small scene (6 impedances and attenuations,
    3 sphere-centre coordinates, 2000 amplitudes) and J itself against the
    oracle's forward-mode gradient of the same paths, with the choice frozen
    and attached."""
    torch, w, g, s, gt = tiny_adj
    got = _gpu_grads(s, w, gt, frozen=frozen)
    ref = oracle.trace_grad(w, g.astype(np.float64), attach_choice=not frozen)
    assert np.count_nonzero(ref["sph"]) == 3 and np.count_nonzero(ref["amp"]) > 100
    _assert_matches_oracle(got, ref, f"tiny frozen={frozen}")


def test_trace_adjoint_record_ranges_and_capture_overflow(oracle, torch_gpu):
    """The tangent passes replay the value pass's record of each path's
    decisions, range by range.  120k scatterers packed in the slab the plane
    wave crosses (x +-10 mm, y +-2 mm, z 1-19 mm) give about eight
    contributing captures a path, so a large share of the paths overflow the
    record's 8 captures and walk the scatterer grid again while the others
    replay their recorded captures; ranges of 333 paths leave a ragged last
    range.  Both range sizes match the oracle's gradient, and each other to
    FP64 summation order."""
    mm = 1e-3
    w = _workload(rays=256)
    rng = np.random.default_rng(5)
    pos = rng.uniform([-10 * mm, -2 * mm, 1 * mm], [10 * mm, 2 * mm, 19 * mm], size=(120_000, 3))
    w = _with_scene(w, scat=np.hstack([pos, rng.normal(size=(120_000, 1))]))
    g = _smooth_adjoint((w.acq.n_tx, w.acq.n_elements, w.acq.n_samples), 27)
    s = _sim(w)
    st = s.trace(stats=True, pulse=False)
    per_path = st["records"] / st["rays"]
    print(f"[adjoint-record] records per path {per_path:.2f}", flush=True)
    assert per_path > 5.0
    gt = torch_gpu.from_numpy(g).cuda()
    ranged = _gpu_grads(s, w, gt, frozen=False, record_paths=333)
    whole = _gpu_grads(s, w, gt, frozen=False)
    ref = oracle.trace_grad(w, g.astype(np.float64), attach_choice=True)
    assert np.count_nonzero(ref["sph"]) == 3 and np.count_nonzero(ref["z"]) >= 3
    _assert_matches_oracle(ranged, ref, "dense slab, ranges of 333 paths")
    _assert_matches_oracle(whole, ref, "dense slab, one range")
    for key in ("z", "sph"):
        a, b = ranged[key].ravel(), whole[key].ravel()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), key


def test_trace_adjoint_matches_oracle_gradient_convex(oracle, torch_gpu):
    w = scenes.convex_probe(_workload(), 20e-3)
    g = _smooth_adjoint((w.acq.n_tx, w.acq.n_elements, w.acq.n_samples), 23)
    s = _sim(w)
    got = _gpu_grads(s, w, torch_gpu.from_numpy(g).cuda(), frozen=False)
    ref = oracle.trace_grad(w, g.astype(np.float64), attach_choice=True)
    assert np.count_nonzero(ref["alpha"]) > 0
    _assert_matches_oracle(got, ref, "convex")


def test_trace_adjoint_matches_oracle_gradient_bone_reduced(oracle, torch_gpu):
    """Bone phantom (60k-triangle tube, three slabs, 50k scatterers), 11
    plane waves, 6 rays per element, linear binning."""
    w = scenes.bone(rays_per_element=6)
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, binning=scenes.LINEAR))
    g = _smooth_adjoint((w.acq.n_tx, w.acq.n_elements, w.acq.n_samples), 24)
    s = _sim(w)
    got = _gpu_grads(s, w, torch_gpu.from_numpy(g).cuda(), frozen=False)
    ref = oracle.trace_grad(w, g.astype(np.float64), attach_choice=True)
    assert np.count_nonzero(ref["z"]) >= 3
    _assert_matches_oracle(got, ref, "bone-reduced")


def test_large_scene_gradient_matches_oracle(oracle, torch_gpu):
    """The differentiable large scene at full size (192 elements, 21 plane
    waves, two 250k-triangle tubes, 4 spheres, 1e6 scatterers, linear
    binning) on a stride sample the oracle can replay (every 8268th ray of
    each (transmit, element) row, 15 rays per row): J, all 6 impedances, all 6
    attenuations, all 12 sphere-centre coordinates (frozen choice) and all
    1e6 amplitude gradients, element by element, against the oracle's
    forward-mode gradient of the same paths."""
    w = scenes.large()
    stride = 8268
    A = w.acq
    g = _smooth_adjoint((A.n_tx, A.n_elements, A.n_samples), 41)
    s = _sim(w)
    print("[adjoint-oracle] large: GPU replay", flush=True)
    got = _gpu_grads(s, w, torch_gpu.from_numpy(g).cuda(), stride=stride, frozen=True)
    print("[adjoint-oracle] large: oracle replay", flush=True)
    ref = oracle.trace_grad(w, g.astype(np.float64), attach_choice=False, ray_stride=stride)
    assert np.count_nonzero(ref["amp"]) >= 150 and np.count_nonzero(ref["alpha"]) >= 3
    _assert_matches_oracle(got, ref, "large")


def test_choice_probability_term_is_unbiased(torch_gpu):
    """Scatterers above a single reflector and no sphere: the impedance of
    the reflector changes only the reflect-or-transmit probability of the
    paths that contribute, so the frozen-choice gradient is exactly zero and
    the full gradient is the score term alone.  Its mean over seeds must
    match common-random-number central differences of the forward data."""
    torch = torch_gpu
    w = _workload(rays=2048, binning=scenes.NEAREST)
    sc = w.scene
    keep = sc.scat[:, 2] < 19.0 * scenes.MM
    w = _with_scene(w, sph=np.zeros((0, 4)), sph_mat=np.zeros((0, 2), np.int32), scat=sc.scat[keep])
    s = _sim(w)
    g = _smooth_adjoint((1, w.acq.n_elements, w.acq.n_samples), 31)
    gt = torch.from_numpy(g).cuda()
    Z = torch.empty(len(w.scene.materials), dtype=torch.float64, device="cuda")
    s.ctx.ur_trace_adjoint(w.seed, gt, Z=Z, frozen_choice=True)
    assert float(Z[1]) == 0.0
    mat0 = w.scene.materials.copy()
    h = 0.2
    gd, fd = [], []
    for k in range(24):
        seed = 9000 + k
        s.ctx.ur_scene_update(mat=mat0)
        s.ctx.ur_trace_adjoint(seed, gt, Z=Z)
        gd.append(float(Z[1]))
        js = []
        for sgn in (1, -1):
            mat = mat0.copy()
            mat[1, 0] += sgn * h
            s.ctx.ur_scene_update(mat=mat)
            s.trace(seed=seed, pulse=False)
            js.append(float((s.ch_raw.double() * gt.double()).sum()))
        fd.append((js[0] - js[1]) / (2 * h))
    s.ctx.ur_scene_update(mat=mat0)
    gd, fd = np.array(gd), np.array(fd)
    d = gd - fd
    se = d.std(ddof=1) / math.sqrt(len(d))
    print(f"[adjoint] score term: grad {gd.mean():.4e} fd {fd.mean():.4e} se {se:.2e}", flush=True)
    assert abs(gd.mean()) > 3 * gd.std(ddof=1) / math.sqrt(len(gd))   # the term is resolved
    assert abs(d.mean()) < 4.5 * se


def test_autograd_envelope_loss(torch_gpu):
    """End to end: envelope loss -> amplitude, attenuation, impedance and
    sphere-centre gradients through the autograd function; the amplitude
    gradient along a random direction matches central differences of the
    GPU forward (the data are linear in the amplitudes before the envelope)."""
    torch = torch_gpu
    from paper_2501_05828_amd.adjoint import simulate_envelope
    w = _workload(rays=256)
    s = _sim(w)
    sc = w.scene
    amp = torch.tensor(sc.scat[:, 3], dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor(sc.materials[:, 1], requires_grad=True)
    Z = torch.tensor(sc.materials[:, 0], requires_grad=True)
    cen = torch.tensor(sc.sph[:, :3], requires_grad=True)
    env_t = simulate_envelope(s, amp, alpha, Z, cen).detach() * 0.9
    env = simulate_envelope(s, amp, alpha, Z, cen)
    loss = 0.5 * ((env.double() - env_t.double()) ** 2).sum()
    loss.backward()
    for t in (amp, alpha, Z, cen):
        assert t.grad is not None and torch.isfinite(t.grad).all()
    assert float(amp.grad.abs().sum()) > 0 and float(alpha.grad.abs().sum()) > 0
    rng = np.random.default_rng(3)
    v = torch.from_numpy(rng.normal(size=len(sc.scat)))
    eps = 1e-3
    ls = []
    with torch.no_grad():
        for sgn in (1, -1):
            e = simulate_envelope(s, amp + sgn * eps * v, alpha, Z, cen)
            ls.append(float((0.5 * (e.double() - env_t.double()) ** 2).sum()))
    fd = (ls[0] - ls[1]) / (2 * eps)
    got = float(amp.grad @ v)
    print(f"[adjoint] autograd amp dir: grad={got:.6e} fd={fd:.6e}", flush=True)
    assert abs(got - fd) <= 2e-3 * abs(fd)


def test_large_scene_gradients_on_64_parameters(torch_gpu):
    """The differentiable large scene at full size (192 elements, 21 plane
    waves, two 250k-triangle tubes, 4 spheres, 1e6 scatterers, linear
    binning), every 96th ray of each (transmit, element) row (5.2e6 rays).
    The replayed FP64 functional J = sum g c equals sum g * ch_raw of the
    forward trace (itself oracle-checked).  64 parameters -- the 6
    attenuations, the 12 sphere-centre coordinates (frozen choice), 40
    scatterer amplitudes and the 6 impedances (frozen choice) -- are checked
    against central differences of J; a step counts only if the forward's
    integer counters and its number of non-empty bins are unchanged at both
    ends.  With 1e6 scatterers, an impedance step as small as 1e-10 MRayl
    already moves some refracted segment across a capture boundary, so the
    impedances are checked with every amplitude set to zero (captures then
    add nothing to J, and their counters are left out of the check)."""
    torch = torch_gpu
    w = scenes.large()
    stride = 96
    s = _sim(w)
    A = w.acq
    g = _smooth_adjoint((A.n_tx, A.n_elements, A.n_samples), 41)
    gt = torch.from_numpy(g).cuda()
    sc = w.scene
    n_mat, n_sph, K = len(sc.materials), len(sc.sph), len(sc.scat)
    mat0, sph0, amp0 = sc.materials.copy(), sc.sph.copy(), sc.scat[:, 3].copy()
    no_capture = ["rays", "segments", "reflect", "transmit", "tir", "direct_hits", "dropped", "term_box",
                  "term_bounce", "term_time", "term_path"]

    def forward_key(keys):
        st = s.trace(stats=True, ray_stride=stride, pulse=False)
        nz = torch.count_nonzero(s.ch_raw).item()
        return ({k: st[k] for k in keys}, nz), float((s.ch_raw.double() * gt.double()).sum())

    last = {}

    def update(mat, sph, amp):
        """Uploads only the arrays that differ from the last upload."""
        arg = {}
        for name, a in (("mat", mat), ("sph", sph), ("scat_amp", amp)):
            if name not in last or last[name] is not a:
                arg[name] = a
                last[name] = a
        if arg:
            s.ctx.ur_scene_update(**arg)

    def replay_J(mat, sph, amp, keys):
        update(mat, sph, amp)
        v = torch.zeros(1, dtype=torch.float64, device="cuda")
        s.ctx.ur_trace_adjoint(w.seed, gt, value=v, ray_stride=stride)
        return float(v.item()), (forward_key(keys)[0] if keys else None)

    def fd(make, h0, key0, keys, tries=5):
        h = h0
        for _ in range(tries):
            jp, kp = replay_J(*make(h), keys)
            jm, km = replay_J(*make(-h), keys)
            if not keys or (kp == key0 and km == key0):
                return (jp - jm) / (2 * h), h
            h *= 0.1
        return None, h

    def gradients(amp, frozen=True):
        update(mat0, sph0, amp)
        Zg = torch.empty(n_mat, dtype=torch.float64, device="cuda")
        al = torch.empty(n_mat, dtype=torch.float64, device="cuda")
        cg = torch.empty((n_sph, 3), dtype=torch.float64, device="cuda")
        ag = torch.empty(K, device="cuda")
        s.ctx.ur_trace_adjoint(w.seed, gt, amp=ag, alpha=al, Z=Zg, sph_center=cg, frozen_choice=frozen,
                               ray_stride=stride)
        return Zg.cpu().numpy(), al.cpu().numpy(), cg.cpu().numpy().ravel(), ag.double().cpu().numpy()

    update(mat0, sph0, amp0)
    key0, jf = forward_key(EXACT_STATS)
    J0, _ = replay_J(mat0, sph0, amp0, None)
    print(f"[adjoint-large] J replay {J0:.9e} forward {jf:.9e} records {key0[0]['records']}", flush=True)
    assert abs(J0 - jf) <= 1e-5 * abs(J0)
    Zg, al, cg, ag = gradients(amp0)
    checked = {"Z": 0, "alpha": 0, "centre": 0, "amp": 0}
    for m in range(n_mat):
        def mk(h, m=m):
            mat = mat0.copy()
            mat[m, 1] += h
            return mat, sph0, amp0
        f, _ = fd(mk, 1e-4, key0, None)   # no decision depends on attenuation
        print(f"[adjoint-large] dJ/dalpha[{m}] gpu {al[m]:.6e} fd {f:.6e}", flush=True)
        assert abs(al[m] - f) <= 1e-5 * max(np.max(np.abs(al)), abs(f)) + 1e-4 * abs(f)
        checked["alpha"] += 1
    for c in range(3 * n_sph):
        def mk(h, c=c):
            sph = sph0.copy()
            sph[c // 3, c % 3] += h
            return mat0, sph, amp0
        f, h = fd(mk, 1e-10, key0, EXACT_STATS, tries=4)
        print(f"[adjoint-large] dJ/dcentre[{c}] gpu {cg[c]:.6e} fd {f} h {h:.1e}", flush=True)
        if f is not None:
            assert abs(cg[c] - f) <= 1e-4 * max(np.max(np.abs(cg)), abs(f))
            checked["centre"] += 1
    nonzero = np.flatnonzero(ag)
    rng = np.random.default_rng(17)
    picks = list(rng.choice(nonzero, size=min(30, len(nonzero)), replace=False))
    picks += list(rng.choice(np.flatnonzero(ag == 0), size=40 - len(picks), replace=False))
    for k in picks:
        def mk(h, k=k):
            amp = amp0.copy()
            amp[k] += h
            return mat0, sph0, amp
        f, _ = fd(mk, 1.0, key0, None)   # J is linear in the amplitudes
        assert abs(ag[k] - f) <= 1e-5 * np.max(np.abs(ag)) + 1e-4 * abs(f), (k, ag[k], f)
        checked["amp"] += 1
    # impedances with the captures silenced
    zero = np.zeros_like(amp0)
    update(mat0, sph0, zero)
    keyz, _ = forward_key(no_capture)
    Zz = gradients(zero)[0]
    for m in range(n_mat):
        def mk(h, m=m):
            mat = mat0.copy()
            mat[m, 0] += h
            return mat, sph0, zero
        f, h = fd(mk, 1e-8 * mat0[m, 0], keyz, no_capture, tries=4)
        print(f"[adjoint-large] dJ/dZ[{m}] (no captures) gpu {Zz[m]:.6e} fd {f} h {h:.1e}", flush=True)
        if f is not None:
            assert abs(Zz[m] - f) <= 1e-4 * max(np.max(np.abs(Zz)), abs(f))
            checked["Z"] += 1
    s.ctx.ur_scene_update(mat=mat0, sph=sph0, scat_amp=amp0)
    print(f"[adjoint-large] checked {checked}", flush=True)
    assert checked["Z"] >= n_mat - 1 and checked["centre"] >= 3 * n_sph - 4
    assert sum(checked.values()) >= 58
