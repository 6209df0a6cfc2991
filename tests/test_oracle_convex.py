"""Pins of the oracle's convex array (Sec. 2.3 "Ray Emission": lateral
elements on an arc of given radius; Sec. 4's convex probe) and of the sector
grid and scan conversion used to display its images.

Each test checks the oracle against geometry or a closed form fixed
independently of its code: element centres on the circle, plane-front
delays, a normal-incidence echo from a concentric spherical mirror, the
transducer-sampling value of one capture, the linear limit of a very large
radius, bilinear reproduction of a bilinear field, and a focused point echo.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

MM = 1e-3


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as o
    return o


def _convex_acq(E=64, pitch=0.3 * MM, radius=20 * MM, **kw):
    w = scenes.tiny()
    return dataclasses.replace(w.acq, n_elements=E, pitch=pitch, radius=radius, **kw)


def test_element_centres_lie_on_the_arc(oracle):
    R = 20 * MM
    acq = _convex_acq(E=65, radius=R)
    g = oracle.element_geometry(acq)
    x, z, s, c = g.T
    # on the circle of radius R about (0, 0, -R), normal = radial unit vector
    assert np.allclose(np.hypot(x, z + R), R, rtol=0, atol=1e-15)
    assert np.allclose(s, x / R, atol=1e-15) and np.allclose(c, (z + R) / R, atol=1e-15)
    assert np.allclose(s ** 2 + c ** 2, 1.0, atol=1e-15)
    # neighbours one arc length `pitch` apart: chord 2 R sin(pitch / 2R)
    chord = np.hypot(np.diff(x), np.diff(z))
    assert np.allclose(chord, 2 * R * math.sin(acq.pitch / (2 * R)), rtol=1e-12)
    # symmetric about the middle element, which touches z = 0 facing +z
    assert np.allclose(x, -x[::-1], atol=1e-18) and np.allclose(z, z[::-1], atol=1e-18)
    assert x[32] == 0.0 and z[32] == 0.0 and c[32] == 1.0
    # a linear array: the usual pitch grid on z = 0, all facing +z
    gl = oracle.element_geometry(dataclasses.replace(acq, radius=0.0))
    assert np.array_equal(gl[:, 0], (np.arange(65) - 32) * acq.pitch)
    assert not gl[:, 1].any() and not gl[:, 2].any() and np.all(gl[:, 3] == 1.0)


def test_convex_delays_follow_the_plane_front(oracle):
    """Each element fires when the steered plane front passes its centre:
    tau_e - k.c_e / c0 is the same for every element, and the earliest
    element fires at 0."""
    acq = _convex_acq(angles=np.deg2rad([-30.0, -4.0, 0.0, 17.0]))
    g = oracle.element_geometry(acq)
    for tx, th in enumerate(acq.angles):
        tau = np.array([oracle.delay(acq, tx, e) for e in range(acq.n_elements)])
        kc = (g[:, 0] * math.sin(th) + g[:, 1] * math.cos(th)) / acq.c0
        assert tau.min() == 0.0
        assert np.ptp(tau - kc) < 1e-20
    # at 0 degrees the front reaches the middle (deepest) element last
    tau0 = np.array([oracle.delay(acq, 2, e) for e in range(acq.n_elements)])
    assert tau0.argmax() in (31, 32) and tau0[0] == tau0[-1] == 0.0


def _mirror_workload(R, D, Z_mirror=1000.0):
    """Water inside a sphere of radius R + D about the centre of curvature;
    the sphere's outside is a near-total reflector."""
    w = scenes.tiny()
    box = np.array([-30 * MM, -20 * MM, -4 * MM, 30 * MM, 20 * MM, 40 * MM])
    mats = np.array([[1.5, 0.0, 1540.0], [Z_mirror, 0.0, 1540.0]])
    sc = scenes.Scene(mats, box, 0, np.zeros((0, 9)), np.zeros((0, 2), np.int32),
                      np.array([[0.0, 0.0, -R, R + D]]), np.array([[1, 0]], np.int32),
                      np.zeros((0, 4)), np.zeros((0, 2), np.int32), np.zeros((0, 4)))
    acq = _convex_acq(radius=R)
    return dataclasses.replace(w, scene=sc, acq=acq)


def test_normal_ray_echoes_back_into_its_element(oracle):
    """A ray leaving the arc along its outward normal meets the concentric
    mirror at normal incidence, returns along itself, lands where it left
    and is recorded by the element it left from at time 2 D / c with its full
    weight (the receive angle to that element's normal is below alpha_m)."""
    R, D, c = 20 * MM, 10 * MM, 1540.0
    w = _mirror_workload(R, D)
    dphi = w.acq.pitch / R
    rays, want = [], []
    for i, (e, u) in enumerate([(0, 0.1), (7, 0.5), (31, 0.93), (32, 0.02), (50, 0.6), (63, 0.9)]):
        ph = (e - 31.5 + u - 0.5) * dphi
        o = (R * math.sin(ph), 0.0, R * math.cos(ph) - R)
        d = (math.sin(ph), 0.0, math.cos(ph))
        rays.append(dict(o=o, d=d, w=0.75, t=1e-6, elem=e, ray=i))
        want.append((e, o))
    ev, st, _ = oracle.trace_rays(w, rays)
    direct = [x for x in ev if x["kind"] == "direct"]
    assert st["reflect"] + st["transmit"] == len(rays)
    assert len(direct) == st["reflect"] >= 4          # R^2 = 0.994 per ray
    for x in direct:
        # the recorded element is the one whose arc holds the origin
        cand = [k for k, (e, o) in enumerate(want) if e == x["elem"]]
        assert len(cand) == 1
        e, o = want[cand[0]]
        assert x["t"] == pytest.approx(1e-6 + 2 * D / c, rel=1e-13)
        assert x["value"] == pytest.approx(0.75, rel=1e-13)
        assert np.allclose(x["pos"], o, atol=1e-12)


def test_transducer_sampling_value_on_a_convex_array(oracle):
    """Homogeneous loss-free water and one scatterer: every record of the
    capture is  w a E A cos(alpha) f_d(alpha) / (4 pi r^2)  at time
    t_q + r / c, r the distance to the drawn element's centre and alpha the
    angle between the reversed arrival direction and that element's normal."""
    R, c = 20 * MM, 1540.0
    w = scenes.tiny()
    box = np.array([-30 * MM, -20 * MM, -4 * MM, 30 * MM, 20 * MM, 40 * MM])
    q = np.array([1.7 * MM, 0.4 * MM, 15 * MM])
    amp = -1.3
    sc = scenes.Scene(np.array([[1.5, 0.0, c]]), box, 0, np.zeros((0, 9)), np.zeros((0, 2), np.int32),
                      np.zeros((0, 4)), np.zeros((0, 2), np.int32), np.zeros((0, 4)), np.zeros((0, 2), np.int32),
                      np.array([[q[0], q[1], q[2], amp]]))
    am, ac = math.radians(20.0), math.radians(60.0)
    acq = _convex_acq(radius=R, alpha_m=am, alpha_c=ac)
    w = dataclasses.replace(w, scene=sc, acq=acq)
    g = oracle.element_geometry(acq)
    o = np.array([q[0], q[1], -1 * MM])
    rays = [dict(o=o, d=(0.0, 0.0, 1.0), w=0.5, t=2e-6, elem=3, ray=i) for i in range(40)]
    ev, st, _ = oracle.trace_rays(w, rays)
    rec = [x for x in ev if x["kind"] == "scatter"]
    assert st["scatter_events"] == 40 and len(rec) == st["nee_cast"] >= 10
    for x in rec:
        e = x["elem"]
        v = g[e, :2] - q[[0, 2]]
        vv = np.array([v[0], -q[1], v[1]])
        r = np.linalg.norm(vv)
        cos_a = -(vv[0] * g[e, 2] + vv[2] * g[e, 3]) / r
        al = math.acos(min(1.0, cos_a))
        fd = 1.0 if al <= am else (ac - al) / (ac - am)
        tq = 2e-6 + (q[2] - o[2]) / c
        area = acq.pitch * acq.elevation
        want = 0.5 * amp * acq.n_elements * area * cos_a * fd / (4 * math.pi * r * r)
        assert x["t"] == pytest.approx(tq + r / c, rel=1e-9)
        assert x["value"] == pytest.approx(want, rel=1e-9)
        assert np.allclose(x["pos"], q, atol=1e-15)


def test_large_radius_reproduces_the_linear_array(oracle):
    """At a radius of 1e9 m the arc is flat to 1e-13 m over the aperture:
    the trace (emission, probe face, direct hits, transducer sampling,
    binning) must reproduce the linear array's, counts exactly."""
    w = scenes.tiny(rays_per_element=256)
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, binning=scenes.LINEAR, alpha_m=math.radians(10.0),
                                                       alpha_c=math.radians(30.0)))
    ch_l, st_l = oracle.trace(w)
    box = np.array(w.scene.box).copy()
    box[2] = -1e-12
    wc = dataclasses.replace(w, scene=dataclasses.replace(w.scene, box=box),
                             acq=dataclasses.replace(w.acq, radius=1e9))
    ch_c, st_c = oracle.trace(wc)
    for k in ("rays", "segments", "reflect", "transmit", "tir", "scatter_events", "nee_zero", "nee_cast",
              "nee_blocked", "direct_hits", "records", "term_box", "term_bounce"):
        assert st_l[k] == st_c[k], k
    assert st_l["direct_hits"] > 0 and st_l["nee_cast"] > 0
    assert np.allclose(ch_c, ch_l, rtol=0, atol=1e-6 * np.abs(ch_l).max())


def test_convex_rejects_a_box_through_the_array(oracle):
    w = scenes.tiny_convex(rays_per_element=4)
    box = np.array(w.scene.box).copy()
    box[2] = -0.5 * MM                     # box top cuts through the array
    with pytest.raises(RuntimeError):
        oracle.trace(dataclasses.replace(w, scene=dataclasses.replace(w.scene, box=box)))


def test_tiny_convex_trace_invariants(oracle):
    w = scenes.tiny_convex(rays_per_element=128)
    ch, st = oracle.trace(w)
    assert st["rays"] == w.acq.n_rays
    assert st["term_box"] + st["term_bounce"] + st["term_time"] + st["term_path"] == st["rays"]
    assert st["records"] == st["direct_hits"] + st["nee_cast"] - st["nee_blocked"] - st["dropped"]
    assert st["direct_hits"] > 0 and st["nee_cast"] > 0 and st["media_mismatch"] == 0


def test_sector_points_closed_form(oracle):
    R = 20 * MM
    g = scenes.Grid(7, 5, -0.4, 0.3, 1 * MM, 30 * MM, sector=True)
    xz = oracle.sector_points(R, g)
    ph = np.repeat(np.linspace(g.x0, g.x1, g.nx), g.nz)
    r = np.tile(np.linspace(g.z0, g.z1, g.nz), g.nx)
    assert np.allclose(np.hypot(xz[:, 0], xz[:, 1] + R), R + r, rtol=1e-14)
    assert np.allclose(np.arctan2(xz[:, 0], xz[:, 1] + R), ph, atol=1e-14)


def test_scan_conversion_reproduces_a_bilinear_field(oracle):
    """Bilinear interpolation is exact for a + b phi + c r + d phi r; outside
    the sector the fill value."""
    R = 20 * MM
    sec = scenes.Grid(33, 41, -0.45, 0.5, 2 * MM, 36 * MM, sector=True)
    ph = np.linspace(sec.x0, sec.x1, sec.nx)[:, None]
    r = np.linspace(sec.z0, sec.z1, sec.nz)[None, :]
    f = lambda p, q: 0.3 + 2.0 * p - 40.0 * q + 15.0 * p * q
    img = f(ph, r)
    cart = scenes.Grid(57, 61, -30 * MM, 30 * MM, -3 * MM, 40 * MM)
    out = oracle.scan_convert(R, sec, img, cart, fill=-7.0)
    xs = np.linspace(cart.x0, cart.x1, cart.nx)[:, None]
    zs = np.linspace(cart.z0, cart.z1, cart.nz)[None, :] + R
    pp, rr = np.arctan2(xs, zs), np.hypot(xs, zs) - R
    inside = (pp >= sec.x0) & (pp <= sec.x1) & (rr >= sec.z0) & (rr <= sec.z1)
    assert inside.sum() > 500 and (~inside).sum() > 500
    assert np.allclose(out[inside], f(pp, rr)[inside], atol=1e-12)
    assert np.all(out[~inside] == -7.0)


def test_convex_das_focuses_point_echo(oracle):
    """An analytic echo of a point (plane front k.p referenced to the first
    element it passes, straight return to each element centre) focuses at
    that point with the full coherent sum."""
    acq = _convex_acq(angles=np.deg2rad([-12.0, 0.0, 8.0]))
    g = oracle.element_geometry(acq)
    E, S = acq.n_elements, acq.n_samples
    x0, z0 = -4.3 * MM, 16.1 * MM
    sig = acq.n_cycles / (2 * math.sqrt(2 * math.log(2)) * acq.f_c)
    tn = (np.arange(S) + 0.5) / acq.f_s
    rf = np.zeros((len(acq.angles), E, S), complex)
    for tx, th in enumerate(acq.angles):
        kc = g[:, 0] * math.sin(th) + g[:, 1] * math.cos(th)
        t_tx = (x0 * math.sin(th) + z0 * math.cos(th) - kc.min()) / acq.c0
        for e in range(E):
            dt = tn - (t_tx + math.hypot(x0 - g[e, 0], z0 - g[e, 1]) / acq.c0)
            rf[tx, e] = np.exp(-dt ** 2 / (2 * sig ** 2)) * np.exp(2j * math.pi * acq.f_c * dt)
    apod = 0.5 - 0.5 * np.cos(2 * np.pi * (np.arange(E) + 0.5) / E)
    v = oracle.das_points(acq, [[x0, z0]], rf)[0]
    full = len(acq.angles) * apod.sum()
    assert math.cos(math.pi / 8) * full * 0.999 <= abs(v) <= full * 1.0001
    xs = x0 + np.linspace(-0.6, 0.6, 13) * MM
    zs = z0 + np.linspace(-0.3, 0.3, 13) * MM
    env = np.abs(oracle.das_points(acq, np.array([[x, z] for x in xs for z in zs]), rf)).reshape(13, 13)
    i, j = np.unravel_index(env.argmax(), env.shape)
    assert abs(xs[i] - x0) <= 0.1 * MM and abs(zs[j] - z0) <= 0.05 * MM


@pytest.mark.parametrize("radius", [0.0, 20 * MM, 50 * MM])
def test_cone_elements_are_exactly_the_hearing_ones(oracle, radius):
    """The cone-restricted element range (linear arrays, and its form for
    convex arrays) against brute force over every element centre: it holds every
    element whose acceptance cone contains the point, and nothing else
    beyond elements at the cut-off to within 1e-7 rad."""
    ac = math.radians(6.0)
    acq = _convex_acq(E=128, pitch=0.45 * MM, radius=radius, alpha_m=math.radians(2.0), alpha_c=ac,
                      element_choice=1)
    g = oracle.element_geometry(acq)
    rng = np.random.default_rng(11)
    n_hit = n_none = 0
    for _ in range(3000):
        q = np.array([rng.uniform(-40, 40) * MM, rng.normal(0, 1.5) * MM, rng.uniform(0.5, 90) * MM])
        v = q[None, :] - np.stack([g[:, 0], np.zeros(len(g)), g[:, 1]], 1)
        cosa = (v[:, 0] * g[:, 2] + v[:, 2] * g[:, 3]) / np.linalg.norm(v, axis=1)
        al = np.arccos(np.clip(cosa, -1, 1))
        heard = np.nonzero(al <= ac)[0]
        r = oracle.cone_elements(acq, q)
        if r is None:
            assert len(heard) == 0 or np.all(np.abs(al[heard] - ac) < 1e-7)
            n_none += 1
            continue
        lo, n = r
        rng_set = np.arange(lo, lo + n)
        assert set(heard) <= set(rng_set)
        extra = np.setdiff1d(rng_set, heard)
        assert np.all(np.abs(al[extra] - ac) < 1e-7), (q, al[extra] - ac)
        n_hit += 1
    assert n_hit > 300 and n_none > 100


@pytest.mark.parametrize("choice", [0, 1])
def test_convex_element_choice_expectation_closed_form(oracle, choice):
    """One scatterer in attenuating water under a convex array: the mean
    recorded contribution equals the closed-form sum over all elements of the
    Eq. 13-weighted, attenuated re-radiation toward each centre (normal of
    each element), for the uniform (weight E) and the cone choice (weight K)
    alike; within 5 standard errors."""
    alpha, c, R = 0.7, 1500.0, 20 * MM
    p = np.array([1.3 * MM, 0.05 * MM, 15 * MM])
    amp = 1.3
    box = np.array([-30 * MM, -20 * MM, -4 * MM, 30 * MM, 20 * MM, 40 * MM])
    sc = scenes.Scene(np.array([[1.5, alpha, c]]), box, 0, np.zeros((0, 9)), np.zeros((0, 2), np.int32),
                      np.zeros((0, 4)), np.zeros((0, 2), np.int32), np.zeros((0, 4)), np.zeros((0, 2), np.int32),
                      np.array([[p[0], p[1], p[2], amp]]))
    acq = _convex_acq(radius=R, alpha_m=math.radians(2.0), alpha_c=math.radians(5.0), element_choice=choice)
    w = dataclasses.replace(scenes.tiny(), scene=sc, acq=acq)
    g = oracle.element_geometry(acq)
    o = np.array([0.3 * MM, 0.0, -1 * MM])
    d = p - o
    d[1] = 0.0
    d /= np.linalg.norm(d)
    n = 3000
    rays = [dict(o=o, d=d, w=2.0, t=1e-6, ray=r, elem=3) for r in range(n)]
    ev, _, _ = oracle.trace_rays(w, rays, cap=4 * n)
    s = np.dot(p - o, d)
    q = o + s * d
    ka = alpha * 5 * 100 * math.log(10) / 20
    want = 0.0
    for k in range(acq.n_elements):
        ce = np.array([g[k, 0], 0.0, g[k, 1]])
        v = q - ce
        r = np.linalg.norm(v)
        cos_a = (v[0] * g[k, 2] + v[2] * g[k, 3]) / r
        al = math.acos(min(1.0, cos_a))
        f = 1.0 if al <= acq.alpha_m else (0.0 if al > acq.alpha_c else (acq.alpha_c - al) / (acq.alpha_c - acq.alpha_m))
        want += 2.0 * math.exp(-ka * (s + r)) * amp * acq.pitch * acq.elevation * cos_a * f / (4 * math.pi * r * r)
    recs = [e["value"] for e in ev if e["kind"] == "scatter"]
    vals = np.array(recs + [0.0] * (n - len(recs)))
    se = vals.std(ddof=1) / math.sqrt(n)
    assert want > 0 and abs(vals.mean() - want) < 5 * se + 1e-15
    if choice == 1:
        assert len(recs) > 0.5 * n
