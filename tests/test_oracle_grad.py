"""Pins of the oracle's forward-mode gradient (or_trace_grad): the
derivative of J = sum over records of g(t) c, g a fixed adjoint of the
binned channel data, with respect to impedances, attenuations, sphere
centres and scatterer amplitudes, along the oracle's own paths.

Each pin compares it with something computed another way:

- its value J equals sum(g * ch_raw) of the oracle's forward trace;
- amplitudes: J is linear in them, so central differences are exact;
- attenuation: no decision depends on it, so central differences of the
  forward trace converge as h^2;
- impedances and sphere centres with the reflect-or-transmit choice frozen:
  central differences of the forward trace at steps small enough that no
  decision changes (every integer counter and the set of non-empty bins
  equal at p - h, p, p + h), through spheres, planes, triangles and a
  convex array, with linear binning (arrival-time derivatives) and nearest
  binning;
- the attached choice probability: per explicit ray, the difference between
  the attached and the frozen gradient equals, for every record after the
  ray's one interface, g(t) c times the derivative of the log-probability
  of the choice taken, that derivative from central differences of the
  pinned Fresnel function (or_interface).
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

MM = 1e-3
COUNTERS = ["rays", "segments", "reflect", "transmit", "tir", "scatter_events", "nee_zero", "nee_cast",
            "nee_blocked", "direct_hits", "records", "dropped", "term_box", "term_bounce", "term_time",
            "term_path"]


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as o
    return o


def _tiny(rays=1024, binning=scenes.LINEAR, convex=False):
    """The tiny scene with its sphere moved under the aperture (centre
    12 mm deep) so that paths meet it; wide receive cone."""
    w = scenes.tiny_convex(rays_per_element=rays) if convex else scenes.tiny(rays_per_element=rays)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45), binning=binning)
    sph = np.array([[1.0e-3, 0.5e-3, 12.0e-3, 3.0e-3]])
    return dataclasses.replace(w, acq=acq, scene=dataclasses.replace(w.scene, sph=sph,
                                                                     sph_mat=np.array([[0, 2]], np.int32)))


def _adjoint(w, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(w.acq.n_tx, w.acq.n_elements, w.acq.n_samples))


def _J(oracle, w, g, stride):
    ch, st = oracle.trace(w, ray_stride=stride)
    return float(np.sum(g * ch)), ({k: st[k] for k in COUNTERS}, np.flatnonzero(ch).tobytes())


def _fd(oracle, w, g, stride, perturb, h, tries=3):
    """Central difference of J with every decision unchanged at both ends
    (the step shrinks until so); None if no step is clean."""
    _, k0 = _J(oracle, w, g, stride)
    for _ in range(tries):
        jp, kp = _J(oracle, perturb(w, h), g, stride)
        jm, km = _J(oracle, perturb(w, -h), g, stride)
        if kp == k0 and km == k0:
            return (jp - jm) / (2 * h)
        h *= 0.1
    return None


def _mat(col, m):
    def perturb(w, h):
        mat = w.scene.materials.copy()
        mat[m, col] += h
        return dataclasses.replace(w, scene=dataclasses.replace(w.scene, materials=mat))
    return perturb


def _centre(j, c):
    def perturb(w, h):
        sph = w.scene.sph.copy()
        sph[j, c] += h
        return dataclasses.replace(w, scene=dataclasses.replace(w.scene, sph=sph))
    return perturb


@pytest.fixture(scope="module")
def tiny_grad(oracle):
    w = _tiny()
    g = _adjoint(w, 21)
    return w, g, oracle.trace_grad(w, g, ray_stride=4)


def test_value_equals_the_forward_functional(oracle, tiny_grad):
    w, g, r = tiny_grad
    ch, st = oracle.trace(w, ray_stride=4)
    assert st["records"] > 100
    assert r["J"] == pytest.approx(float(np.sum(g * ch)), rel=1e-12)


def test_amplitude_gradient_is_exact(oracle, tiny_grad):
    w, g, r = tiny_grad
    ga = r["amp"]
    assert np.count_nonzero(ga) > 50
    a0 = w.scene.scat[:, 3].copy()
    rng = np.random.default_rng(3)
    dirs = [rng.normal(size=len(a0))]
    for k in np.argsort(-np.abs(ga))[:3]:
        e = np.zeros(len(a0))
        e[k] = 1.0
        dirs.append(e)
    for v in dirs:
        def perturb(ww, h, v=v):
            return dataclasses.replace(ww, scene=dataclasses.replace(
                ww.scene, scat=np.column_stack([ww.scene.scat[:, :3], a0 + h * v])))
        fd = _fd(oracle, w, g, 4, perturb, 1.0, tries=1)
        assert fd is not None and float(ga @ v) == pytest.approx(fd, rel=1e-9, abs=1e-12 * np.abs(ga).max())


def test_attenuation_gradient(oracle, tiny_grad):
    w, g, r = tiny_grad
    for m in range(len(w.scene.materials)):
        fd = _fd(oracle, w, g, 4, _mat(1, m), 1e-4, tries=1)
        assert fd is not None
        assert r["alpha"][m] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(r["alpha"]).max())


def test_impedance_gradient_frozen_choice(oracle, tiny_grad):
    w, g, r = tiny_grad
    scale = np.abs(r["z"]).max()
    for m in range(len(w.scene.materials)):
        fd = _fd(oracle, w, g, 4, _mat(0, m), 1e-7)
        assert fd is not None
        assert abs(r["z"][m] - fd) <= 1e-5 * scale, (m, r["z"][m], fd)


def test_sphere_centre_gradient_frozen_choice(oracle, tiny_grad):
    w, g, r = tiny_grad
    scale = np.abs(r["sph"]).max()
    assert scale > 0
    for c in range(3):
        fd = _fd(oracle, w, g, 4, _centre(0, c), 1e-9)
        assert fd is not None
        assert abs(r["sph"][0, c] - fd) <= 1e-5 * scale, (c, r["sph"][0, c], fd)


def test_nearest_binning_has_no_time_term(oracle):
    """With nearest binning the data are piecewise constant in arrival time:
    the frozen derivative is that of the values alone."""
    w = _tiny(binning=scenes.NEAREST)
    g = _adjoint(w, 22)
    r = oracle.trace_grad(w, g, ray_stride=4)
    for m in range(len(w.scene.materials)):
        fd = _fd(oracle, w, g, 4, _mat(0, m), 1e-7)
        assert fd is not None and abs(r["z"][m] - fd) <= 1e-5 * np.abs(r["z"]).max()
    for c in range(3):
        fd = _fd(oracle, w, g, 4, _centre(0, c), 1e-9)
        assert fd is not None and abs(r["sph"][0, c] - fd) <= 1e-5 * np.abs(r["sph"]).max()


def test_gradient_through_a_triangle_mesh(oracle):
    """A refracting plane at 8 mm over a closed cube mesh (12 triangles,
    Z 2.5): the impedances bend the rays that then meet the triangles, so
    the triangle distances' derivatives enter."""
    from tests.test_oracle_pins import cube_mesh, homogeneous
    tri = cube_mesh((-6 * MM, -6 * MM, 12 * MM), (6 * MM, 6 * MM, 22 * MM))
    rng = np.random.default_rng(7)
    scat = np.column_stack([rng.uniform([-15 * MM, -15 * MM, 1 * MM], [15 * MM, 15 * MM, 38 * MM], (800, 3)),
                            rng.normal(size=800)])
    sc = homogeneous(mats=[[1.5, 0.5, 1540.0], [1.62, 0.7, 1580.0], [2.5, 1.0, 1540.0]],
                     planes=[[0, 0, 1, 8 * MM]], pln_mat=[[1, 0]], tri=tri, tri_mat=[[1, 2]] * 12, scat=scat)
    w = scenes.tiny(rays_per_element=512)
    w = dataclasses.replace(w, scene=sc, acq=dataclasses.replace(w.acq, alpha_m=math.radians(10),
                                                                 alpha_c=math.radians(45), binning=scenes.LINEAR))
    g = _adjoint(w, 23)
    r = oracle.trace_grad(w, g, ray_stride=2)
    scale = np.abs(r["z"]).max()
    assert scale > 0
    for m in range(3):
        fd = _fd(oracle, w, g, 2, _mat(0, m), 1e-7)
        assert fd is not None and abs(r["z"][m] - fd) <= 1e-5 * scale, (m, r["z"][m], fd)
        fd = _fd(oracle, w, g, 2, _mat(1, m), 1e-4, tries=1)
        assert r["alpha"][m] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(r["alpha"]).max())


def test_gradient_on_a_convex_array(oracle):
    """Convex array (the array's cylinder as the absorbing face, element
    normals in the receive angle)."""
    w = _tiny(convex=True)
    g = _adjoint(w, 24)
    r = oracle.trace_grad(w, g, ray_stride=4)
    assert np.abs(r["alpha"]).max() > 0
    for m in range(len(w.scene.materials)):
        fd = _fd(oracle, w, g, 4, _mat(0, m), 1e-7)
        assert fd is not None and abs(r["z"][m] - fd) <= 1e-5 * np.abs(r["z"]).max()
    for c in range(3):
        fd = _fd(oracle, w, g, 4, _centre(0, c), 1e-9)
        assert fd is not None and abs(r["sph"][0, c] - fd) <= 1e-5 * max(np.abs(r["sph"]).max(), 1e-30)


def _tent_g(g, t, fs):
    x = t * fs - 0.5
    n0 = math.floor(x)
    f = x - n0
    S = len(g)
    g0 = g[n0] if 0 <= n0 < S else 0.0
    g1 = g[n0 + 1] if 0 <= n0 + 1 < S else 0.0
    return (1 - f) * g0 + f * g1


def test_attached_choice_adds_the_score_of_the_choice(oracle):
    """Explicit rays onto the 20 mm reflector of the tiny scene (no sphere):
    each meets one interface, reflects up to the array or transmits into
    the reflector, and records captures before and after it.  For every ray,
    attached minus frozen gradient of each impedance = sum over the records
    after the interface of g(t) c d log P/dZ, with P = R or 1 - R at its
    incidence angle and dP/dZ from central differences of or_interface."""
    w = scenes.tiny(rays_per_element=1)
    w = dataclasses.replace(w, scene=dataclasses.replace(w.scene, sph=np.zeros((0, 4)),
                                                         sph_mat=np.zeros((0, 2), np.int32)),
                            acq=dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45),
                                                    binning=scenes.LINEAR))
    g = _adjoint(w, 25)
    Z = w.scene.materials[:, 0]
    rng = np.random.default_rng(9)
    checked = 0
    for r in range(200):
        # near-normal incidence, so that reflected rays return into the aperture as direct hits
        th, ph = math.acos(rng.uniform(0.999, 1.0)), rng.uniform(0, 2 * math.pi)
        d = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
        ray = dict(o=[rng.uniform(-8, 8) * MM, rng.uniform(-0.5, 0.5) * MM, 0.0], d=d, w=1.0, ray=r,
                   elem=r % 64)
        a = oracle.trace_grad(w, g, attach_choice=True, rays=[ray])
        f = oracle.trace_grad(w, g, attach_choice=False, rays=[ray])
        ev, _, _ = oracle.trace_rays(w, [ray], cap=2000)
        iface = [e for e in ev if e["kind"] in ("reflect", "transmit")]
        assert len(iface) <= 1
        if not iface:
            assert np.allclose(a["z"], f["z"], rtol=0, atol=1e-300)
            continue
        refl = iface[0]["kind"] == "reflect"
        after = sum(_tent_g(g[0, e["elem"]], e["t"], w.acq.f_s) * e["value"]
                    for e in ev if e["kind"] in ("direct", "scatter") and e["seg"] >= 1)
        for m in (0, 1):
            h = 1e-6
            Rs = []
            for sgn in (1, -1):
                zz = Z.copy()
                zz[m] += sgn * h
                _, _, R = oracle.interface(np.array(d), np.array([0.0, 0.0, 1.0]), zz[1], zz[0], 0.5)
                Rs.append(R if refl else 1.0 - R)
            _, _, R0 = oracle.interface(np.array(d), np.array([0.0, 0.0, 1.0]), Z[1], Z[0], 0.5)
            P0 = R0 if refl else 1.0 - R0
            score = (Rs[0] - Rs[1]) / (2 * h) / P0
            want = after * score
            got = a["z"][m] - f["z"][m]
            assert abs(got - want) <= 1e-6 * abs(want) + 1e-12 * max(abs(a["z"][m]), 1e-300), (r, m, got, want)
        checked += after != 0.0
    assert checked > 40


def test_gradient_through_rough_boundaries(oracle):
    """Rough boundaries (Eq. 12, GGX; reflector roughness 0.3, sphere 0.5)
    with their echoes received by direct hits only: the microfacet normal
    follows the sphere's normal for the same random numbers and the weight
    factor is differentiated with it; central differences of the forward
    trace with every decision (including absorptions at the rough
    boundaries) unchanged."""
    w = _tiny()
    w = dataclasses.replace(w, scene=dataclasses.replace(w.scene, rough=np.array([0.0, 0.3, 0.5])),
                            acq=dataclasses.replace(w.acq, rough_direct_only=1))
    g = _adjoint(w, 31)
    r = oracle.trace_grad(w, g, ray_stride=4)
    ch, st = oracle.trace(w, ray_stride=4)
    assert st["term_rough"] > 100 and r["J"] == pytest.approx(float(np.sum(g * ch)), rel=1e-12)
    for m in range(3):
        fd = _fd(oracle, w, g, 4, _mat(0, m), 1e-7)
        assert fd is not None and abs(r["z"][m] - fd) <= 1e-5 * np.abs(r["z"]).max(), (m, r["z"][m], fd)
        fd = _fd(oracle, w, g, 4, _mat(1, m), 1e-4, tries=1)
        assert r["alpha"][m] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(r["alpha"]).max())
    for c in range(3):
        fd = _fd(oracle, w, g, 4, _centre(0, c), 1e-9)
        assert fd is not None and abs(r["sph"][0, c] - fd) <= 1e-5 * np.abs(r["sph"]).max(), (c, r["sph"][0, c], fd)
    # with transducer sampling at the rough boundaries: not supported
    w2 = dataclasses.replace(w, acq=dataclasses.replace(w.acq, rough_direct_only=0))
    with pytest.raises(RuntimeError, match="-3"):
        oracle.trace_grad(w2, g, ray_stride=4)
