"""Pins of the FP64 oracle against physics, closed forms and brute force.

Every test here checks the oracle against something other than itself:
closed forms of the paper's equations, geometric invariants, analytically
known intersections, statistical expectations, or values in tests/golden
(computed from the paper's stated parameters with plain math).
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

MM = 1e-3


def homogeneous(alpha=0.5, c=1540.0, Z=1.5, box=(-20, -20, 0, 20, 20, 40), planes=(), pln_mat=(), mats=None,
                tri=None, tri_mat=None, sph=None, sph_mat=None, scat=None):
    mats = np.array(mats if mats is not None else [[Z, alpha, c]], float)
    return scenes.Scene(
        materials=mats, box=np.array(box, float) * MM, top_medium=0,
        tri=np.zeros((0, 9)) if tri is None else np.asarray(tri, float).reshape(-1, 9),
        tri_mat=np.zeros((0, 2), np.int32) if tri_mat is None else np.asarray(tri_mat, np.int32).reshape(-1, 2),
        sph=np.zeros((0, 4)) if sph is None else np.asarray(sph, float).reshape(-1, 4),
        sph_mat=np.zeros((0, 2), np.int32) if sph_mat is None else np.asarray(sph_mat, np.int32).reshape(-1, 2),
        pln=np.asarray(planes, float).reshape(-1, 4), pln_mat=np.asarray(pln_mat, np.int32).reshape(-1, 2),
        scat=np.zeros((0, 4)) if scat is None else np.asarray(scat, float).reshape(-1, 4))


def with_scene(scene, **acq_kw):
    w = scenes.tiny()
    acq = dataclasses.replace(w.acq, **acq_kw) if acq_kw else w.acq
    return dataclasses.replace(w, scene=scene, acq=acq)


def cube_mesh(lo, hi):
    """Closed axis-aligned cube as 12 outward-wound triangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    V = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], float)
    F = [(0, 2, 1), (0, 3, 2), (4, 5, 6), (4, 6, 7), (0, 1, 5), (0, 5, 4),
         (2, 3, 7), (2, 7, 6), (1, 2, 6), (1, 6, 5), (0, 4, 7), (0, 7, 3)]
    return np.array([np.concatenate([V[a], V[b], V[c]]) for a, b, c in F])


# ------------------------------------------------------------------ Philox
def test_philox_known_answers(oracle):
    """The generator equals the published Philox4x32-10 definition on its
    known-answer vectors (tests/golden/philox_kat.json, with its source)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert oracle.philox(ctr, key) == [int(x, 16) for x in v["out"]]


def test_philox_uniformity_and_avalanche(oracle):
    """Counter-based RNG: uniform words, and one flipped counter or key bit
    changes about half the output bits."""
    n = 20000
    words = np.array([oracle.philox([i, 7, 3 | (1 << 16), 11], [0x5EED0001, 0]) for i in range(n)], np.uint64)
    u = (words.astype(np.float64) + 0.5) / 2 ** 32
    counts, _ = np.histogram(u.ravel(), bins=64, range=(0, 1))
    exp = u.size / 64
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 120, chi2                        # 63 dof, p ~ 1e-5
    flips = []
    rng = np.random.default_rng(0)
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        base = oracle.philox(c, k)
        word, bit = int(rng.integers(0, 6)), int(rng.integers(0, 32))
        c2, k2 = list(c), list(k)
        if word < 4:
            c2[word] ^= 1 << bit
        else:
            k2[word - 4] ^= 1 << bit
        out = oracle.philox(c2, k2)
        flips.append(sum(bin(a ^ b).count("1") for a, b in zip(base, out)))
    assert 60 < np.mean(flips) < 68


# ------------------------------------------------------- emission map / Eq. 6
def test_hemisphere_map_is_unit_and_equal_area(oracle):
    """The square-to-hemisphere map has constant Jacobian 2*pi (equal area):
    every one of the 32x32 cells subtends 2*pi/1024 sr."""
    rng = np.random.default_rng(1)
    h = 1e-6
    for a, b in rng.uniform(0.02, 0.98, size=(300, 2)):
        d = oracle.hemisphere(a, b)
        assert abs(np.linalg.norm(d) - 1) < 1e-12 and d[2] >= 0
        if min(abs(abs(2 * a - 1) - abs(2 * b - 1)), abs(2 * a - 1), abs(2 * b - 1)) < 1e-4:
            continue                               # the map's fold lines
        da = (oracle.hemisphere(a + h, b) - oracle.hemisphere(a - h, b)) / (2 * h)
        db = (oracle.hemisphere(a, b + h) - oracle.hemisphere(a, b - h)) / (2 * h)
        assert abs(np.linalg.norm(np.cross(da, db)) - 2 * np.pi) < 1e-5
    # cell solid angle by quadrature of the Jacobian over one cell
    cell = 5 * 32 + 17
    ia, ib = cell % 32, cell // 32
    m = 24
    tot = 0.0
    for i in range(m):
        for j in range(m):
            a = (ia + (i + 0.5) / m) / 32
            b = (ib + (j + 0.5) / m) / 32
            da = (oracle.hemisphere(a + h, b) - oracle.hemisphere(a - h, b)) / (2 * h)
            db = (oracle.hemisphere(a, b + h) - oracle.hemisphere(a, b - h)) / (2 * h)
            tot += np.linalg.norm(np.cross(da, db)) / (32 * m) ** 2
    assert abs(tot - 2 * np.pi / 1024) < 1e-9


def test_uniform_emission_moments(oracle):
    """Uniform hemisphere: E[cos theta] = 1/2, E[d_x] = E[d_y] = 0."""
    g = (np.arange(200) + 0.5) / 200
    D = np.array([oracle.hemisphere(a, b) for a in g for b in g])
    assert abs(D[:, 2].mean() - 0.5) < 1e-4
    assert abs(D[:, 0].mean()) < 1e-9 and abs(D[:, 1].mean()) < 1e-9


# ------------------------------------------------------------ Eq. 13
def test_receive_directivity_table(oracle):
    am, ac = math.radians(2), math.radians(6)
    assert oracle.directivity(0.0, am, ac) == 1.0
    assert oracle.directivity(am, am, ac) == 1.0
    assert abs(oracle.directivity(math.radians(4), am, ac) - 0.5) < 1e-12
    assert oracle.directivity(-math.radians(4), am, ac) == pytest.approx(0.5)
    assert oracle.directivity(ac, am, ac) == pytest.approx(0.0, abs=1e-15)
    assert oracle.directivity(math.radians(7), am, ac) == 0.0
    # the paper's setting alpha_m = alpha_c = 2 deg is a hard cut-off
    a2 = math.radians(2)
    assert oracle.directivity(a2 * 0.999, a2, a2) == 1.0
    assert oracle.directivity(a2 * 1.001, a2, a2) == 0.0


# ------------------------------------------------------ Eqs. 7-11
def _rand_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_reflection_law(oracle):
    rng = np.random.default_rng(2)
    for _ in range(200):
        n = _rand_unit(rng)
        d = _rand_unit(rng)
        refl, out, R = oracle.interface(d, n, 1.5, 7.8, 0.0)   # y = 0 < R always reflects
        assert refl
        assert abs(np.linalg.norm(out) - 1) < 1e-12
        assert abs(np.dot(out, n) + np.dot(d, n)) < 1e-12        # angle in = angle out
        assert abs(np.linalg.det(np.array([d, n, out]))) < 1e-12  # coplanar
        assert np.linalg.norm(out - d) > 0 or abs(np.dot(d, n)) < 1e-15


def test_snell_and_fresnel(oracle, golden):
    rng = np.random.default_rng(3)
    for zf, zb in [(1.5, 7.8), (7.8, 1.5), (1.5, 3.0), (1.62, 1.45)]:
        for _ in range(200):
            n = _rand_unit(rng)
            d = _rand_unit(rng)
            refl, out, R = oracle.interface(d, n, zf, zb, 1.0 - 1e-12)  # y ~ 1: transmit unless TIR
            z1, z2 = (zf, zb) if np.dot(d, n) < 0 else (zb, zf)
            eta = z1 / z2
            sin_i = np.linalg.norm(np.cross(d, n))
            if eta * sin_i > 1:                                    # total internal reflection
                assert refl and R == 1.0
                continue
            assert not refl
            assert abs(np.linalg.norm(out) - 1) < 1e-12
            sin_t = np.linalg.norm(np.cross(out, n))
            assert abs(sin_t - eta * sin_i) < 1e-10                # Snell with eta = Z1/Z2
            assert np.sign(np.dot(out, n)) == np.sign(np.dot(d, n))  # continues to the far side
            assert abs(np.linalg.det(np.array([d, n, out]))) < 1e-12
            assert 0 <= R <= 1
    for case in golden["interfaces"]:
        n = np.array([0, 0, 1.0])
        _, _, R = oracle.interface(-n, n, case["z2"], case["z1"], 0.5)   # front = z2 side? ray hits from front
        _, _, R2 = oracle.interface(n * 1.0, n, case["z2"], case["z1"], 0.5)
        assert abs(R - case["R_normal"]) < 1e-12 and abs(R2 - case["R_normal"]) < 1e-12
        assert abs((1 - R) - case["T_normal"]) < 1e-12


def test_total_internal_reflection_onset(oracle, golden):
    for case in golden["critical"]:
        th = math.radians(case["critical_deg"])
        n = np.array([0, 0, 1.0])
        for dth, tir in [(-1e-6, False), (1e-6, True)]:
            a = th + dth
            d = np.array([math.sin(a), 0, -math.cos(a)])          # travels from the front (z1) side
            refl, out, R = oracle.interface(d, n, case["z1"], case["z2"], 1.0 - 1e-12)
            assert (R == 1.0) == tir


# ------------------------------------------------------ intersections
def test_closest_hit_matches_analytic_cube(oracle):
    """A triangulated closed cube inside a larger box: the brute-force
    closest hit from inside equals the analytic slab exit of the cube."""
    lo, hi = np.array([-5, -4, 6.0]) * MM, np.array([6, 5, 15.0]) * MM
    tri = cube_mesh(lo, hi)
    sc = homogeneous(tri=tri, tri_mat=[[0, 0]] * 12)
    rng = np.random.default_rng(4)
    for _ in range(300):
        o = rng.uniform(lo + 1e-4, hi - 1e-4)
        d = _rand_unit(rng)
        t_exp = min(((hi[i] if d[i] > 0 else lo[i]) - o[i]) / d[i] for i in range(3) if d[i] != 0)
        pid, t = oracle.closest_hit(sc, o, d)
        assert pid < 12 and abs(t - t_exp) < 1e-12


def test_crossing_parity_closed_mesh(oracle):
    """A segment between two points crosses a closed surface an even number
    of times iff both points are on the same side."""
    lo, hi = np.array([-5, -4, 6.0]) * MM, np.array([6, 5, 15.0]) * MM
    tri = cube_mesh(lo, hi)
    sph = [[0.0, 0.0, 30 * MM, 4 * MM]]
    sc = homogeneous(tri=tri, tri_mat=[[0, 0]] * 12, sph=sph, sph_mat=[[0, 0]])
    rng = np.random.default_rng(5)
    for _ in range(300):
        p = rng.uniform([-15 * MM, -15 * MM, 1 * MM], [15 * MM, 15 * MM, 39 * MM], size=(2, 3))
        v = p[1] - p[0]
        L = np.linalg.norm(v)
        n = len(oracle.crossings(sc, p[0], v / L, L))
        inside = [bool(np.all(q > lo) and np.all(q < hi)) for q in p]
        in_s = [np.linalg.norm(q - np.array(sph[0][:3])) < sph[0][3] for q in p]
        assert n % 2 == (inside[0] != inside[1]) ^ (in_s[0] != in_s[1])


def test_sphere_and_plane_hits(oracle):
    sc = homogeneous(planes=[[0, 0, 1, 20 * MM]], pln_mat=[[0, 0]], sph=[[3 * MM, 1 * MM, 10 * MM, 2 * MM]],
                     sph_mat=[[0, 0]])
    pid, t = oracle.closest_hit(sc, [3 * MM, 1 * MM, 0.0], [0, 0, 1.0])
    assert pid == 0 and abs(t - 8 * MM) < 1e-15               # sphere first (id 0), front surface
    pid, t = oracle.closest_hit(sc, [3 * MM, 1 * MM, 10 * MM], [0, 0, 1.0])
    assert pid == 0 and abs(t - 2 * MM) < 1e-15               # from the centre: far root
    pid, t = oracle.closest_hit(sc, [-10 * MM, 0.0, 0.0], [0, 0.6, 0.8])
    assert pid == 1 and abs(t - 25 * MM) < 1e-15              # plane at 20 mm, cos = 0.8
    pid, t = oracle.closest_hit(sc, [-10 * MM, 0.0, 20 * MM], [0, 0.6, 0.8], skip=1)
    assert pid == 2                                            # plane excluded -> box exit


# ------------------------------------------------------ whole-path pins
def _ray_id_with(oracle, seed, want_reflect, R, seg=0, tx=0, e=0):
    for r in range(1000):
        y = (oracle.philox([r, e | (tx << 16), seg | (1 << 16), 0], [seed & 0xFFFFFFFF, seed >> 32])[0] + 0.5) / 2 ** 32
        if (y < R) == want_reflect:
            return r
    raise AssertionError


def test_echo_time_and_attenuation_planar_reflector(oracle, golden):
    """One ray straight down onto the 20 mm reflector, reflected branch:
    arrival 2d/c, bin floor(2d/c fs), amplitude exp(-alpha f 2d)."""
    g = golden["echo"]
    sc = homogeneous(alpha=0.5, planes=[[0, 0, 1, 20 * MM]], pln_mat=[[1, 0]],
                     mats=[[1.5, 0.5, 1540.0], [7.8, 0.5, 1540.0]])
    w = with_scene(sc)
    R = golden["interfaces"][1]["R_normal"]
    r = _ray_id_with(oracle, w.seed, True, R)
    x = 0.15 * MM                                           # centre of element 32
    ev, st, hist = oracle.trace_rays(w, [dict(o=[x, 0, 0], d=[0, 0, 1], w=1.0, t=0.0, ray=r)], with_hist=True)
    rec = [e for e in ev if e["kind"] == "direct"]
    assert len(rec) == 1
    assert abs(rec[0]["t"] - g["t_echo"]) < 1e-15
    assert rec[0]["elem"] == 32
    assert abs(rec[0]["value"] - g["amplitude_factor"]) < 1e-14
    assert hist[0, 32, g["bin"]] == pytest.approx(g["amplitude_factor"], rel=1e-14)
    assert np.count_nonzero(hist) == 1
    # transmitted branch: absorbed by the box, nothing recorded
    r2 = _ray_id_with(oracle, w.seed, False, R)
    ev2, _, _ = oracle.trace_rays(w, [dict(o=[x, 0, 0], d=[0, 0, 1], ray=r2)])
    assert not [e for e in ev2 if e["kind"] in ("direct", "scatter")]
    assert [e for e in ev2 if e["kind"] == "transmit"]


def test_attenuation_matched_impedance_slab(oracle):
    """Equal impedances never reflect; the weight after crossing two media is
    exactly exp(-sum_m alpha_m f d_m) and the time sum_m d_m / c_m."""
    mats = [[1.5, 0.5, 1540.0], [1.5, 3.0, 1600.0]]
    sc = homogeneous(planes=[[0, 0, 1, 12 * MM]], pln_mat=[[1, 0]], mats=mats)
    w = with_scene(sc)
    ev, _, _ = oracle.trace_rays(w, [dict(o=[0, 0, 0], d=[0, 0, 1], w=1.0, ray=5)])
    assert [e["kind"] for e in ev] == ["transmit", "end"]
    end = ev[-1]
    ln10 = math.log(10)
    expected = math.exp(-(0.5 * 5 * 1.2 + 3.0 * 5 * 2.8) * ln10 / 20)
    assert abs(end["value"] / expected - 1) < 1e-13
    assert abs(end["t"] - (12 * MM / 1540 + 28 * MM / 1600)) < 1e-18


def _tent(x, n_samples):
    """The linear reconstruction filter by its definition: sample m is
    centred at (m + 1/2)/fs and receives the fraction 1 - |t fs - (m + 1/2)|
    (clipped at zero) of an arrival at t."""
    m = np.arange(n_samples)
    return np.maximum(0.0, 1.0 - np.abs(x - (m + 0.5)))


@pytest.mark.parametrize("x", [0.2, 0.5, 0.8, 1.5, 1.8, 1000.5, 1000.8, 1001.499, 2046.5, 2046.8, 2047.3,
                               2047.5, 2047.9])
def test_linear_binning_tent_weights(oracle, x):
    """LINEAR binning (the differentiable workload's reconstruction filter):
    an explicit ray arriving head-on at element 32 at t = x / fs puts
    (1 - f) w into sample n and f w into sample n + 1, with n + 1/2 + f = x
    (the tent centred on each sample), including the first and the last
    sample of the record; an arrival at or after S / fs records nothing."""
    sc = homogeneous(alpha=0.0)
    w = with_scene(sc, binning=scenes.LINEAR)
    fs, S, c = w.acq.f_s, w.acq.n_samples, 1540.0
    z0 = 5 * MM
    t0 = x / fs - z0 / c
    ev, st, hist = oracle.trace_rays(w, [dict(o=[0.15 * MM, 0, z0], d=[0, 0, -1], w=0.75, t=t0, ray=3)],
                                     with_hist=True)
    rec = [e for e in ev if e["kind"] == "direct"]
    assert len(rec) == 1 and rec[0]["elem"] == 32 and rec[0]["value"] == 0.75
    assert rec[0]["t"] == pytest.approx(x / fs, rel=1e-14)
    expected = 0.75 * _tent(rec[0]["t"] * fs, S)
    assert np.allclose(hist[0, 32], expected, rtol=0, atol=1e-12)
    assert np.count_nonzero(hist[0, :32]) == 0 and np.count_nonzero(hist[0, 33:]) == 0
    # the two weights: (1 - f) into n, f into n + 1
    n = int(math.floor(x - 0.5))
    f = (x - 0.5) - n
    if 0 <= n < S:
        assert hist[0, 32, n] == pytest.approx(0.75 * (1 - f), abs=1e-12)
    if 0 <= n + 1 < S:
        assert hist[0, 32, n + 1] == pytest.approx(0.75 * f, abs=1e-12)
    assert hist.sum() == pytest.approx(0.75 * ((1 - f) * (0 <= n < S) + f * (0 <= n + 1 < S)), abs=1e-12)
    # NEAREST binning of the same arrival: all of it in floor(x)
    w0 = with_scene(sc)
    _, _, h0 = oracle.trace_rays(w0, [dict(o=[0.15 * MM, 0, z0], d=[0, 0, -1], w=0.75, t=t0, ray=3)],
                                 with_hist=True)
    assert h0[0, 32, int(math.floor(x))] == 0.75 and np.count_nonzero(h0) == 1


def test_arrival_at_the_end_of_the_record_is_dropped(oracle):
    sc = homogeneous(alpha=0.0)
    for binning in (scenes.NEAREST, scenes.LINEAR):
        w = with_scene(sc, binning=binning)
        x = w.acq.n_samples + 0.25
        t0 = x / w.acq.f_s - 5 * MM / 1540.0
        ev, st, hist = oracle.trace_rays(w, [dict(o=[0.15 * MM, 0, 5 * MM], d=[0, 0, -1], t=t0, ray=3)],
                                         with_hist=True)
        # the time window ends the ray before its direct hit
        assert st["term_time"] == 1 and st["direct_hits"] == 0 and st["records"] == 0
        assert np.count_nonzero(hist) == 0
        # just inside the window: recorded
        t1 = (w.acq.n_samples - 0.25) / w.acq.f_s - 5 * MM / 1540.0
        _, st1, h1 = oracle.trace_rays(w, [dict(o=[0.15 * MM, 0, 5 * MM], d=[0, 0, -1], t=t1, ray=3)],
                                       with_hist=True)
        assert st1["direct_hits"] == 1 and st1["records"] == 1 and h1[0, 32, -1] > 0


def test_path_length_limit_clips_the_last_segment(oracle):
    """A ray whose path would exceed max_path (0.2 m, Sec. 4) ends exactly
    at 0.2 m of path: after a matched boundary at 20 mm (never reflects) it
    stops at depth 0.2 m with time 0.02/c0 + 0.18/c1 and weight
    exp(-k0 0.02 - k1 0.18), k_m = alpha_m ln10/20 f_c in Np per metre."""
    mats = [[1.5, 0.5, 1540.0], [1.5, 2.0, 1500.0]]
    sc = homogeneous(planes=[[0, 0, 1, 20 * MM]], pln_mat=[[1, 0]], mats=mats, box=(-20, -20, 0, 20, 20, 300))
    w = with_scene(sc, n_samples=8192, max_path=0.2)
    ev, st, _ = oracle.trace_rays(w, [dict(o=[0, 0, 0], d=[0, 0, 1], w=1.0, ray=9)])
    assert [e["kind"] for e in ev] == ["transmit", "end"]
    end = ev[-1]
    assert end["id"] == -3 and end["seg"] == 1
    assert end["pos"][2] == pytest.approx(0.2, abs=1e-15) and end["pos"][0] == 0.0
    k = lambda a: a * math.log(10) / 20 * 5.0 * 100.0       # dB/(cm MHz) at 5 MHz -> Np/m
    assert end["value"] == pytest.approx(math.exp(-k(0.5) * 0.02 - k(2.0) * 0.18), rel=1e-13)
    assert end["t"] == pytest.approx(0.02 / 1540.0 + 0.18 / 1500.0, rel=1e-14)
    assert st["term_path"] == 1 and st["term_box"] == 0 and st["segments"] == 2
    # a shorter limit clips the first segment instead
    w2 = with_scene(sc, n_samples=8192, max_path=0.015)
    ev2, st2, _ = oracle.trace_rays(w2, [dict(o=[0, 0, 0], d=[0, 0, 1], w=1.0, ray=9)])
    assert [e["kind"] for e in ev2] == ["end"] and ev2[0]["pos"][2] == pytest.approx(0.015, abs=1e-15)
    assert st2["term_path"] == 1 and st2["segments"] == 1


@pytest.mark.parametrize("bounces", [2, 3])
def test_bounce_limit_ends_the_ray_at_the_next_interface(oracle, bounces):
    """At most B interface interactions (Sec. 2.3's interaction limit, 10 in
    Sec. 4): three matched planes at 10, 20, 30 mm.  With B = 2 the ray is
    transmitted twice and ends on reaching the third plane (two interactions
    logged, term_bounce); with B = 3 it crosses all three and leaves through
    the box."""
    mats = [[1.5, 0.5, 1540.0], [1.5, 0.5, 1500.0], [1.5, 0.5, 1560.0], [1.5, 0.5, 1520.0]]
    planes = [[0, 0, 1, 10 * MM], [0, 0, 1, 20 * MM], [0, 0, 1, 30 * MM]]
    sc = homogeneous(planes=planes, pln_mat=[[1, 0], [2, 1], [3, 2]], mats=mats)
    w = with_scene(sc, max_bounces=bounces)
    ev, st, _ = oracle.trace_rays(w, [dict(o=[0, 0, 0], d=[0, 0, 1], w=1.0, ray=4)])
    kinds = [e["kind"] for e in ev]
    if bounces == 2:
        assert kinds == ["transmit", "transmit", "end"]
        assert ev[-1]["id"] == -4 and ev[-1]["seg"] == 2
        assert ev[-1]["pos"][2] == pytest.approx(30 * MM, abs=1e-15)
        assert ev[-1]["t"] == pytest.approx(10 * MM / 1540 + 10 * MM / 1500 + 10 * MM / 1560, rel=1e-14)
        assert st["term_bounce"] == 1 and st["transmit"] == 2 and st["segments"] == 3
    else:
        assert kinds == ["transmit", "transmit", "transmit", "end"]
        assert ev[-1]["id"] == -1 and ev[-1]["pos"][2] == pytest.approx(40 * MM, abs=1e-15)
        assert st["term_bounce"] == 0 and st["term_box"] == 1 and st["segments"] == 4


def test_oblique_refraction_follows_snell_through_trace(oracle):
    mats = [[1.5, 0.0, 1540.0], [1.8, 0.0, 1540.0]]
    sc = homogeneous(planes=[[0, 0, 1, 10 * MM]], pln_mat=[[1, 0]], mats=mats)
    w = with_scene(sc)
    th = math.radians(25)
    d = [math.sin(th), 0, math.cos(th)]
    ev, _, _ = oracle.trace_rays(w, [dict(o=[-5 * MM, 0, 0], d=d, ray=r) for r in range(40)], cap=1000)
    trans = [e for e in ev if e["kind"] == "transmit"]
    ends = [e for e in ev if e["kind"] == "end"]
    assert trans
    # the transmitted ray leaves the box; its exit point fixes the refracted angle
    for e_t in trans:
        end = next(x for x in ends if x["t"] > e_t["t"] and x["seg"] == 1)
        p0, p1 = np.array(e_t["pos"]), np.array(end["pos"])
        v = (p1 - p0) / np.linalg.norm(p1 - p0)
        assert abs(math.hypot(v[0], v[1]) - (1.5 / 1.8) * math.sin(th)) < 1e-12
        break


def test_reflected_fraction_matches_fresnel(oracle, golden):
    """Over many independent draws the reflect-or-transmit choice reflects
    with probability A_r^2 (binomial 5-sigma band)."""
    sc = homogeneous(alpha=0.0, planes=[[0, 0, 1, 20 * MM]], pln_mat=[[1, 0]],
                     mats=[[1.5, 0.0, 1540.0], [7.8, 0.0, 1540.0]])
    w = with_scene(sc)
    n = 4000
    ev, _, _ = oracle.trace_rays(w, [dict(o=[0, 0, 0], d=[0, 0, 1], ray=r) for r in range(n)], cap=4 * n)
    refl = sum(1 for e in ev if e["kind"] == "reflect")
    R = golden["interfaces"][1]["R_normal"]
    assert abs(refl / n - R) < 5 * math.sqrt(R * (1 - R) / n)


def test_single_scatterer_closed_form(oracle):
    """Homogeneous medium, one scatterer on an explicit ray: contribution and
    arrival time in closed form (isotropic re-radiation toward the chosen
    element's centre, element solid angle A cos(alpha)/r^2 over 4 pi, divided
    by the 1/E choice probability, attenuation along both legs)."""
    alpha, c = 0.7, 1500.0
    p = np.array([1.2 * MM, 0.05 * MM, 15 * MM])
    amp = -1.7
    sc = homogeneous(alpha=alpha, c=c, scat=[[*p, amp]])
    w = with_scene(sc, alpha_m=math.pi / 2, alpha_c=math.pi / 2)
    acq = w.acq
    o = np.array([0.3 * MM, 0.0, 0.0])
    d = p - o
    d[1] = 0.0
    d /= np.linalg.norm(d)
    ev, _, _ = oracle.trace_rays(w, [dict(o=o, d=d, w=2.0, t=1e-6, ray=9, elem=3)])
    rec = [e for e in ev if e["kind"] == "scatter"]
    assert len(rec) == 1
    s = np.dot(p - o, d)
    x = oracle.philox([9, 3, 0 | (2 << 16), 0], [w.seed & 0xFFFFFFFF, w.seed >> 32])[0]
    er = (x * acq.n_elements) >> 32
    assert rec[0]["elem"] == er
    q = o + s * d
    ce = np.array([(er - (acq.n_elements - 1) / 2) * acq.pitch, 0, 0])
    r = np.linalg.norm(ce - q)
    cos_a = q[2] / r
    ka = alpha * 5 * 100 * math.log(10) / 20
    expected = (2.0 * math.exp(-ka * (s + r)) * amp * acq.n_elements * acq.pitch * acq.elevation * cos_a
                / (4 * math.pi * r * r))
    assert abs(rec[0]["value"] / expected - 1) < 1e-12
    assert abs(rec[0]["t"] - (1e-6 + (s + r) / c)) < 1e-18


def test_shadow_ray_transmission_product(oracle):
    """A secondary ray crossing one slab boundary at normal incidence carries
    1 - A_r^2 of the pressure and the delays of both media."""
    mats = [[1.5, 0.0, 1540.0], [3.0, 0.0, 1600.0]]
    p = np.array([0.15 * MM, 0.0, 18 * MM])
    sc = homogeneous(planes=[[0, 0, 1, 10 * MM]], pln_mat=[[1, 0]], mats=mats, scat=[[*p, 1.0]])
    w = with_scene(sc, alpha_m=math.pi / 2, alpha_c=math.pi / 2)
    # start below the boundary in medium 1, ray along x through the scatterer
    o = p - np.array([3 * MM, 0, 0])
    ev, _, _ = oracle.trace_rays(w, [dict(o=o, d=[1, 0, 0], w=1.0, ray=r, medium=1) for r in range(64)], cap=2000)
    recs = [e for e in ev if e["kind"] == "scatter"]
    assert recs
    T = 1 - ((3.0 - 1.5) / 4.5) ** 2
    acq = w.acq
    for rc in recs:
        er = rc["elem"]
        ce = np.array([(er - (acq.n_elements - 1) / 2) * acq.pitch, 0, 0])
        r = np.linalg.norm(ce - p)
        cos_a = p[2] / r
        # path below the boundary: 8 mm / cos_a at 1600, above: 10 mm / cos_a at 1540
        t_exp = 3 * MM / 1600 + (8 * MM / 1600 + 10 * MM / 1540) / cos_a
        assert abs(rc["t"] - t_exp) < 1e-15
        eta = 3.0 / 1.5
        sin_i = math.sqrt(1 - cos_a ** 2)
        ct = math.sqrt(1 - eta ** 2 * sin_i ** 2)
        A = (3.0 * cos_a - 1.5 * ct) / (3.0 * cos_a + 1.5 * ct)
        expected = acq.n_elements * acq.pitch * acq.elevation * cos_a / (4 * math.pi * r * r) * (1 - A * A)
        assert abs(rc["value"] / expected - 1) < 1e-12
    assert abs(T - (1 - (1.5 / 4.5) ** 2)) < 1e-15


def test_emission_weights_mirror_statistics(oracle):
    """Near-total reflector at depth D, no attenuation: the direct-hit sum per
    transmit estimates pi sin^2(alpha_m) (uniform emission, weight
    cos(theta)/(N p)); every arrival is at or after 2D/c."""
    D = 6 * MM
    sc = homogeneous(alpha=0.0, planes=[[0, 0, 1, D]], pln_mat=[[1, 0]],
                     mats=[[1.5, 0.0, 1540.0], [1.5e9, 0.0, 1540.0]], box=(-60, -60, 0, 60, 60, 40))
    am = math.radians(10)
    w = with_scene(sc, alpha_m=am, alpha_c=am, elevation=40 * MM, max_bounces=1)
    w = w.with_rays(1024)
    ch, st = oracle.trace(w)
    total = ch.sum()
    expected = math.pi * math.sin(am) ** 2
    # fraction of the hemisphere inside the cone ~ 1 - cos(am); relative std ~ 1/sqrt(count)
    n_hit = st["direct_hits"]
    assert n_hit > 500
    assert abs(total / expected - 1) < 5 / math.sqrt(n_hit)
    first = np.nonzero(ch[0].any(0))[0][0]
    assert first >= math.floor(2 * D / 1540 * w.acq.f_s)


def test_learned_emission_mirror_statistics(oracle):
    """The same mirror with a peaked emission-cell table (cell probability
    q, p(omega) = q 1024 / (2 pi)): the 1/p weighting keeps the direct-hit
    sum at pi sin^2(alpha_m) (Eq. 4 with a non-uniform p_t).  The recorded
    |c| histogram sums to the channel data (every contribution is positive
    here) and lies only in cells that contain directions inside the cone."""
    D = 6 * MM
    sc = homogeneous(alpha=0.0, planes=[[0, 0, 1, D]], pln_mat=[[1, 0]],
                     mats=[[1.5, 0.0, 1540.0], [1.5e9, 0.0, 1540.0]], box=(-60, -60, 0, 60, 60, 40))
    am = math.radians(10)
    w = with_scene(sc, alpha_m=am, alpha_c=am, elevation=40 * MM, max_bounces=1).with_rays(512)
    i, j = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    q = 1.0 + 9.0 * np.exp(-((i - 15.5) ** 2 + (j - 15.5) ** 2) / (2 * 4.0 ** 2))
    q = (q / q.sum()).ravel()
    E = w.acq.n_elements
    pdf = np.tile(q.astype(np.float32), (1, E, 1))
    cdf = np.cumsum(pdf.astype(np.float64), -1).astype(np.float32)
    cdf[..., -1] = 1.0
    ch, st, hist = oracle.trace(w, pdf=pdf, cdf=cdf, rec_hist=True)
    n_hit = st["direct_hits"]
    assert n_hit > 500
    expected = math.pi * math.sin(am) ** 2
    assert abs(ch.sum() / expected - 1) < 5 / math.sqrt(n_hit)
    assert abs(hist.sum() / ch.sum() - 1) < 1e-12
    for cell in np.flatnonzero(hist.sum((0, 1))):
        a0, b0 = (cell % 32) / 32.0, (cell // 32) / 32.0
        th = min(math.acos(oracle.hemisphere(a0 + da / 32.0, b0 + db / 32.0)[2])
                 for da in np.linspace(0, 1, 6) for db in np.linspace(0, 1, 6))
        assert th <= am + 1e-9, (cell, th)


# ------------------------------------------------------ pulse (Eq. 14)
def test_pulse_taps_closed_form(oracle, golden):
    g = golden["pulse"]
    w = scenes.tiny()
    K, h = oracle.pulse_taps(w.acq)
    assert K == g["half_taps"] == 51
    m = np.arange(-K, K + 1)
    t = m / w.acq.f_s
    env = np.abs(h)
    # Gaussian envelope with the stated FWHM: |h| = 2^(-(2t/FWHM)^2)
    assert np.allclose(env, 2.0 ** (-(2 * t / g["fwhm_s"]) ** 2), rtol=0, atol=1e-15)
    # the real part is the paper's sin(2 pi f_c t) times the window (Eq. 14)
    assert np.allclose(h.real, np.sin(2 * np.pi * g["f_c"] * t) * env, atol=1e-15)
    assert abs(h[K] - (-1j)) < 1e-15


def test_pulse_impulse_response(oracle):
    w = scenes.tiny()
    acq = w.acq
    raw = np.zeros((1, 2, acq.n_samples))
    raw[0, 1, 700] = 2.0
    raw[0, 0, 3] = 1.0                                       # near the start: truncated
    rf = oracle.pulse(acq, raw)
    K, h = oracle.pulse_taps(acq)
    assert np.allclose(rf[0, 1, 700 - K:700 + K + 1], 2.0 * h, atol=1e-15)
    assert np.count_nonzero(np.abs(rf[0, 1]) > 0) == 2 * K + 1
    assert np.allclose(rf[0, 0, :3 + K + 1], h[K - 3:], atol=1e-15)
    # linearity
    raw2 = np.random.default_rng(0).normal(size=raw.shape)
    assert np.allclose(oracle.pulse(acq, raw + 3 * raw2), rf + 3 * oracle.pulse(acq, raw2), atol=1e-12)


# ------------------------------------------------------ delays and DAS
def test_plane_wave_delays(oracle):
    """Steering delays make the element wavelets meet on a tilted plane: the
    arrival time tau_e + (distance along the steered direction) is the same
    for every element, and the first-firing element has zero delay."""
    w = scenes.bone(rays_per_element=1)
    acq = w.acq
    E = acq.n_elements
    xe = (np.arange(E) - (E - 1) / 2) * acq.pitch
    for tx, th in enumerate(acq.angles):
        tau = np.array([oracle.delay(acq, tx, e) for e in range(E)])
        assert tau.min() == pytest.approx(0.0, abs=1e-18)
        u = np.array([math.sin(th), 0, math.cos(th)])
        P = 0.05 * u
        arrive = tau + (np.dot(P, u) - xe * u[0]) / acq.c0     # plane-wave arrival along u
        assert np.ptp(arrive) < 1e-17
        if th > 0:
            assert np.argmin(tau) == 0
        if th < 0:
            assert np.argmin(tau) == E - 1


def _synthetic_point_rf(acq, x0, z0):
    """Analytic echo of a point at (x0, z0) for every transmit and element."""
    E, S = acq.n_elements, acq.n_samples
    xe = (np.arange(E) - (E - 1) / 2) * acq.pitch
    sig = acq.n_cycles / (2 * math.sqrt(2 * math.log(2)) * acq.f_c)
    tn = (np.arange(S) + 0.5) / acq.f_s
    rf = np.zeros((len(acq.angles), E, S), complex)
    for tx, th in enumerate(acq.angles):
        # arrival of the steered plane wave at the point, referenced to the first-firing element
        xref = xe[0] if math.sin(th) >= 0 else xe[-1]
        t_tx = ((x0 - xref) * math.sin(th) + z0 * math.cos(th)) / acq.c0
        for e in range(E):
            t_rt = t_tx + math.hypot(x0 - xe[e], z0) / acq.c0
            dt = tn - t_rt
            rf[tx, e] = np.exp(-dt ** 2 / (2 * sig ** 2)) * np.exp(2j * math.pi * acq.f_c * dt)
    return rf


def test_das_focuses_point_echo(oracle):
    w = scenes.tiny()
    acq = dataclasses.replace(w.acq, angles=np.deg2rad([-6.0, 0.0, 9.0]))
    x0, z0 = 2.1 * MM, 17.3 * MM
    rf = _synthetic_point_rf(acq, x0, z0)
    E = acq.n_elements
    apod = 0.5 - 0.5 * np.cos(2 * np.pi * (np.arange(E) + 0.5) / E)
    v = oracle.das_points(acq, [[x0, z0]], rf)[0]
    # linear interpolation of a carrier at 8 samples per period keeps at least cos(pi/8) of it
    full = len(acq.angles) * apod.sum()
    assert math.cos(math.pi / 8) * full * 0.999 <= abs(v) <= full * 1.0001
    # the envelope peaks at the scatterer on a fine local grid
    xs = x0 + np.linspace(-0.6, 0.6, 13) * MM
    zs = z0 + np.linspace(-0.3, 0.3, 13) * MM
    pts = np.array([[x, z] for x in xs for z in zs])
    env = np.abs(oracle.das_points(acq, pts, rf)).reshape(13, 13)
    i, j = np.unravel_index(env.argmax(), env.shape)
    assert abs(xs[i] - x0) <= 0.1 * MM and abs(zs[j] - z0) <= 0.05 * MM


def test_das_grid_matches_points_and_envelope(oracle):
    w = scenes.tiny()
    acq = w.acq
    g = dataclasses.replace(w.grid, nx=9, nz=11)
    rf = _synthetic_point_rf(acq, 0.0, 20 * MM)
    iq = oracle.das(acq, g, rf)
    xs = np.linspace(g.x0, g.x1, g.nx)
    zs = np.linspace(g.z0, g.z1, g.nz)
    pts = np.array([[x, z] for x in xs for z in zs])
    assert np.allclose(iq.ravel(), oracle.das_points(acq, pts, rf), rtol=1e-14, atol=1e-14)
    env, bm = oracle.envelope(iq, 90.0)
    assert np.allclose(env, np.abs(iq), rtol=1e-15)
    assert bm.max() == 0.0 and bm.min() >= -90.0
    pos = np.where(env > 0, env, np.inf)
    k = np.unravel_index(pos.argmin(), env.shape)
    assert bm[k] == max(-90.0, 20 * math.log10(env[k] / env.max()))
    assert np.all(bm[env == 0] == -90.0)


def test_full_trace_tiny_invariants(oracle):
    """Whole tiny workload: records never precede the shallowest possible
    echo, nothing lands outside the record window, stats add up."""
    w = scenes.tiny()
    ch, st = oracle.trace(w)
    assert st["rays"] == w.acq.n_rays
    assert st["records"] == st["direct_hits"] + st["nee_cast"] - st["nee_blocked"] - (
        st["dropped"])
    assert st["term_box"] + st["term_bounce"] + st["term_time"] + st["term_path"] == st["rays"]
    assert st["media_mismatch"] == 0
    # deterministic in the seed, different for another seed
    ch2, _ = oracle.trace(w, n_threads=3)
    assert np.allclose(ch, ch2, rtol=1e-12, atol=1e-20)
    ch3, _ = oracle.trace(w, seed=w.seed + 1)
    assert not np.allclose(ch, ch3)


# ---------------------------------------------------- rough interfaces (Eq. 12)

@pytest.mark.parametrize("alpha", [0.05, 0.3, 0.5, 1.0, 2.0])
def test_ggx_distribution_is_normalised(oracle, alpha):
    """Eq. 12 as printed is a density of microfacet normals projected on the
    macro surface: the integral of D(h) (n.h) over the hemisphere is 1."""
    from scipy.integrate import quad
    val, _ = quad(lambda th: oracle.ggx_d(alpha, math.cos(th)) * math.cos(th) * math.sin(th), 0.0, math.pi / 2,
                  limit=400, points=[math.atan(alpha)])
    assert abs(2.0 * math.pi * val - 1.0) < 1e-8


def test_ggx_onb_is_orthonormal_and_right_handed(oracle):
    rng = np.random.default_rng(21)
    ns = rng.normal(size=(200, 3))
    ns = np.vstack([ns, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0], [1.0, 0.0, -0.0], [1e-9, 0.0, -1.0]]])
    for n in ns:
        n = n / np.linalg.norm(n)
        t, b = oracle.onb(n)
        assert abs(t @ n) < 1e-14 and abs(b @ n) < 1e-14 and abs(t @ b) < 1e-14
        assert abs(t @ t - 1) < 1e-14 and abs(b @ b - 1) < 1e-14
        assert np.allclose(np.cross(t, b), n, atol=1e-14)


@pytest.mark.parametrize("alpha", [0.2, 0.7])
def test_ggx_sampler_follows_the_density(oracle, alpha):
    """Sampled microfacet normals have P(theta_h <= th) = tan^2 th / (alpha^2 +
    tan^2 th) (the integral of D(h) (n.h) of Eq. 12 over the cap), a uniform
    azimuth, unit length, and the same law about any macro normal."""
    from scipy import stats
    rng = np.random.default_rng(5)
    xi = rng.random((6000, 2))
    n = np.array([0.3, -0.5, 0.8])
    n /= np.linalg.norm(n)
    t, b = oracle.onb(n)
    hs = np.array([oracle.ggx_sample(n, alpha, a, c) for a, c in xi])
    assert np.allclose(np.linalg.norm(hs, axis=1), 1.0, atol=1e-14)
    th = np.arccos(np.clip(hs @ n, -1, 1))
    cdf = lambda x: np.tan(x) ** 2 / (alpha ** 2 + np.tan(x) ** 2)
    assert stats.kstest(th, cdf).pvalue > 1e-3
    ph = np.mod(np.arctan2(hs @ b, hs @ t), 2 * np.pi) / (2 * np.pi)
    assert stats.kstest(ph, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("alpha", [0.2, 0.6, 1.0])
@pytest.mark.parametrize("theta_deg", [0.0, 30.0, 60.0, 80.0])
def test_ggx_smith_masking_projected_area(oracle, alpha, theta_deg):
    """The Smith masking G1 and D satisfy the projected-area identity
    G1(o) * integral of max(0, o.m) D(m) dm = o.n (visible microfacet area
    seen from o equals the macro surface's), by 2-D quadrature."""
    from scipy.integrate import dblquad
    th_o = math.radians(theta_deg)
    o = np.array([math.sin(th_o), 0.0, math.cos(th_o)])

    def f(ph, th):
        m = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        return max(0.0, o @ m) * oracle.ggx_d(alpha, math.cos(th)) * math.sin(th)

    val, _ = dblquad(f, 0.0, math.pi / 2, 0.0, 2 * math.pi, epsabs=1e-10, epsrel=1e-8)
    assert abs(oracle.ggx_g1(alpha, math.cos(th_o)) * val - math.cos(th_o)) < 2e-6


def test_rough_interface_smooth_limit(oracle):
    """At roughness 1e-13 the rough boundary reproduces Eqs. 7-11 at the
    macro normal: the same choice, the same direction, weight factor 1."""
    rng = np.random.default_rng(8)
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        zf, zb = rng.uniform(1.0, 8.0, size=2)
        y, x1, x2 = rng.random(3)
        k, od, R, wf = oracle.interface_rough(d, n, zf, zb, 1e-13, y, x1, x2)
        refl, od0, R0 = oracle.interface(d, n, zf, zb, y)
        if abs(y - R0) < 1e-6:
            continue
        assert k == int(refl)
        assert np.allclose(od, od0, atol=1e-8) and abs(R - R0) < 1e-8 and abs(wf - 1.0) < 1e-8


@pytest.mark.parametrize("alpha,theta_deg", [(0.3, 0.0), (0.3, 50.0), (0.8, 30.0), (0.8, 70.0)])
def test_rough_matched_interface_mean_weight(oracle, alpha, theta_deg):
    """Through a matched boundary (Z1 = Z2: no reflection, no bending) the
    weight factor |i.h| G1(i) G1(o) / (|i.n| |h.n|) averaged over microfacets
    drawn with density D(h) (n.h) equals G1(i), by the projected-area identity;
    Monte Carlo within 5 standard errors."""
    th = math.radians(theta_deg)
    d = np.array([math.sin(th), 0.0, -math.cos(th)])
    n = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(13)
    xi = rng.random((40000, 2))
    w = np.empty(len(xi))
    for i, (a, c) in enumerate(xi):
        k, od, R, wf = oracle.interface_rough(d, n, 1.5, 1.5, alpha, 0.5, a, c)
        assert k in (0, -1)
        if k == 0:
            assert np.allclose(od, d, atol=1e-10)
        w[i] = wf if k == 0 else 0.0
    want = oracle.ggx_g1(alpha, math.cos(th))
    assert abs(w.mean() - want) < 5 * w.std() / math.sqrt(len(w)) + 1e-12


# ------------------------------------------- element choice of transducer sampling

def test_cone_element_choice_is_unbiased_and_lowers_variance(oracle):
    """Choosing the receiving element uniformly among those whose centre the
    capture point's acceptance cone can reach (weight K) instead of among all
    E (weight E) leaves every expectation unchanged: both estimators average
    the same Eq. 13-weighted sum over elements.  Paired over seeds (the
    primary paths are the same in both modes), the difference of a fixed
    linear functional of the channel data has mean zero; the cone choice has
    the smaller variance.  The functional skips the first 300 samples (under
    5.8 mm round trip): captures within millimetres of the face give
    contributions growing as 1/r^2, with unbounded variance in either mode."""
    w = scenes.tiny(rays_per_element=512)
    w = dataclasses.replace(w, acq=dataclasses.replace(w.acq, alpha_m=math.radians(4), alpha_c=math.radians(10)))
    wc = dataclasses.replace(w, acq=dataclasses.replace(w.acq, element_choice=scenes.ELEMENT_CONE))
    rng = np.random.default_rng(2)
    r = rng.normal(size=(1, w.acq.n_elements, w.acq.n_samples))
    r[:, :, :300] = 0.0
    fu, fc = [], []
    for seed in range(12):
        a, su = oracle.trace(w, seed=1000 + seed)
        b, sc = oracle.trace(wc, seed=1000 + seed)
        assert su["segments"] == sc["segments"] and su["direct_hits"] == sc["direct_hits"]
        assert sc["nee_cast"] > su["nee_cast"]
        fu.append(float((a * r).sum()))
        fc.append(float((b * r).sum()))
    fu, fc = np.array(fu), np.array(fc)
    diff = fu - fc
    assert abs(diff.mean()) < 4.0 * diff.std(ddof=1) / math.sqrt(len(diff))
    assert fc.var() < fu.var()


@pytest.mark.parametrize("choice", [0, 1])
def test_element_choice_expectation_closed_form(oracle, choice):
    """One scatterer on explicit rays whose element draws differ (ray ids):
    the mean recorded contribution equals the closed-form sum over all
    elements of the Eq. 13-weighted, attenuated re-radiation toward each
    centre, for the uniform choice (weight E) and the cone choice (weight K)
    alike; within 5 standard errors."""
    alpha, c = 0.7, 1500.0
    p = np.array([1.0 * MM, 0.05 * MM, 15 * MM])
    amp = 1.3
    sc = homogeneous(alpha=alpha, c=c, scat=[[*p, amp]])
    w = with_scene(sc, alpha_m=math.radians(2), alpha_c=math.radians(5), element_choice=choice)
    acq = w.acq
    o = np.array([0.3 * MM, 0.0, 0.0])
    d = p - o
    d[1] = 0.0
    d /= np.linalg.norm(d)
    n = 3000
    rays = [dict(o=o, d=d, w=2.0, t=1e-6, ray=r, elem=3) for r in range(n)]
    ev, _, _ = oracle.trace_rays(w, rays, cap=4 * n)
    # closed form: sum over every element of its contribution
    s = np.dot(p - o, d)
    q = o + s * d
    ka = alpha * 5 * 100 * math.log(10) / 20
    want = 0.0
    for k in range(acq.n_elements):
        ce = np.array([(k - (acq.n_elements - 1) / 2) * acq.pitch, 0, 0])
        r = np.linalg.norm(ce - q)
        al = math.acos(q[2] / r)
        f = 1.0 if al <= acq.alpha_m else (0.0 if al > acq.alpha_c else (acq.alpha_c - al) / (acq.alpha_c - acq.alpha_m))
        want += 2.0 * math.exp(-ka * (s + r)) * amp * acq.pitch * acq.elevation * (q[2] / r) * f / (4 * math.pi * r * r)
    recs = [e["value"] for e in ev if e["kind"] == "scatter"]
    vals = np.array(recs + [0.0] * (n - len(recs)))
    se = vals.std(ddof=1) / math.sqrt(n)
    assert want > 0 and abs(vals.mean() - want) < 5 * se + 1e-15
    if choice == 1:
        assert len(recs) > 0.5 * n      # most cone draws land on a receiving element


# ------------------------------------------------ synthetic-aperture acquisition

def test_synthetic_aperture_sums_to_the_unsteered_plane_wave(oracle):
    """Element-by-element transmits drawn with transmit 0's counters: their
    channel data summed over the emitting element is the 0-degree plane-wave
    trace (every delay zero), path by path."""
    w = scenes.tiny(rays_per_element=256)
    pw, spw = oracle.trace(w)
    sa, ssa = oracle.trace(scenes.synthetic_aperture(w))
    assert sa.shape == (w.acq.n_elements, w.acq.n_elements, w.acq.n_samples)
    for k in ("rays", "segments", "reflect", "transmit", "records", "direct_hits", "nee_cast"):
        assert spw[k] == ssa[k], k
    assert np.allclose(sa.sum(0), pw[0], rtol=1e-12, atol=1e-12 * np.abs(pw).max())


def test_synthesis_with_whole_sample_delays_is_the_steered_trace(oracle):
    """At the steering angle whose delays are whole samples per element
    (sin theta = c0 / (pitch fs)) the synthesised plane wave equals the
    steered plane-wave trace."""
    w = scenes.tiny(rays_per_element=256)
    acq = w.acq
    th = math.asin(acq.c0 / (acq.pitch * acq.f_s))
    for ang in (th, -th):
        ws = dataclasses.replace(w, acq=dataclasses.replace(acq, angles=np.array([ang])))
        pw, _ = oracle.trace(ws)
        sa, _ = oracle.trace(scenes.synthetic_aperture(w))
        syn = oracle.synthesize(acq, sa, [ang])
        assert np.allclose(syn, pw, rtol=1e-9, atol=1e-9 * np.abs(pw).max()), ang


def test_synthesis_fractional_shift_closed_form(oracle):
    """One impulse in element 5's data moves by its delay tau fs = 5 pitch
    sin(theta) fs / c0 samples, split between the two neighbouring samples
    in proportion (linear interpolation)."""
    w = scenes.tiny()
    acq = w.acq
    E, S = acq.n_elements, acq.n_samples
    sa = np.zeros((E, E, S))
    sa[5, 7, 100] = 2.0
    ang = math.radians(3.0)
    out = oracle.synthesize(acq, sa, [ang])
    sh = 5 * acq.pitch * math.sin(ang) * acq.f_s / acq.c0
    i0 = math.floor(100 + sh)
    f = 100 + sh - i0
    want = np.zeros(S)
    want[i0] = 2.0 * (1 - f)
    want[i0 + 1] = 2.0 * f
    assert np.allclose(out[0, 7], want, atol=1e-14)
    assert not out[0, np.arange(E) != 7].any()
