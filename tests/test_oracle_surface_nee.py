"""Pins of transducer sampling at rough boundaries (the paper's Sec. 2.3:
secondary rays are sent towards an element centre at every boundary
interaction before the boundary's own draw; with a rough, GGX boundary they
carry the boundary's scattering toward that direction).

- The density of directions the rough-boundary sampler produces integrates,
  over the sphere, to the fraction of draws it does not absorb (checked by
  quadrature against the sampler itself): this fixes the Jacobians of the
  reflected and refracted half-vector maps and the Fresnel lobe choice.
- Its scattering toward a direction, divided by that density, is the weight
  the sampler gives the same direction.
- Transducer sampling balanced with the direct hits leaves the expected
  channel data unchanged: the per-element received signal with it equals
  the direct-hits-only signal within the statistical error, while most of
  the signal now comes from the secondary rays.  This holds too when a
  smooth boundary (matched or mismatched in impedance) lies between the
  rough boundary and the array, where the primary ray reaches the array only
  through that boundary and a straight secondary ray would count the same
  echo a second time.
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


def _sphere_grid(n_theta=300, n_phi=600):
    th = (np.arange(n_theta) + 0.5) * math.pi / n_theta
    ph = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    T, Pp = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(Pp), np.sin(T) * np.sin(Pp), np.cos(T)], -1).reshape(-1, 3)
    dw = (np.sin(T) * (math.pi / n_theta) * (2 * math.pi / n_phi)).ravel()
    return dirs, dw


@pytest.mark.parametrize("z1,z2,alpha,theta_deg", [(1.5, 7.8, 0.5, 0.0), (1.5, 7.8, 0.5, 40.0),
                                                  (1.5, 1.7, 0.6, 25.0), (1.7, 1.5, 0.6, 50.0)])
def test_rough_direction_density_integrates_to_the_kept_fraction(oracle, z1, z2, alpha, theta_deg):
    n = np.array([0.0, 0.0, 1.0])
    th = math.radians(theta_deg)
    d = np.array([math.sin(th), 0.0, -math.cos(th)])            # arriving from the +n side
    wi = -d
    rng = np.random.default_rng(1)
    m = 40000
    kept = 0
    for _ in range(m):
        r = oracle.interface_rough(d, n, z1, z2, alpha, rng.random(), rng.random(), rng.random())
        kept += r[0] >= 0
    frac = kept / m
    se = math.sqrt(frac * (1 - frac) / m)
    dirs, dw = _sphere_grid()
    total = 0.0
    for o, w in zip(dirs[::1], dw[::1]):
        _, p = oracle.rough_fcos(wi, n, z1, z2, alpha, o)
        total += p * w
    assert abs(total - frac) < 5 * se + 3e-3, (total, frac)


def test_rough_scattering_over_density_is_the_sampler_weight(oracle):
    rng = np.random.default_rng(2)
    n = np.array([0.0, 0.0, 1.0])
    checked = 0
    for z1, z2, alpha in [(1.5, 7.8, 0.3), (1.5, 1.6, 0.7), (1.6, 1.5, 1.2)]:
        for _ in range(300):
            th = math.acos(rng.uniform(0.1, 1.0))
            ph = rng.uniform(0, 2 * math.pi)
            d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th)])
            refl, od, R, wf = oracle.interface_rough(d, n, z1, z2, alpha, rng.random(), rng.random(), rng.random())
            if refl < 0:
                continue
            fc, p = oracle.rough_fcos(-d, n, z1, z2, alpha, od)
            assert p > 0 and fc > 0
            assert fc / p == pytest.approx(wf, rel=1e-9)
            checked += 1
    assert checked > 600


def _rough_floor_workload(alpha, direct_only, rays_per_element=512):
    """Water over a rough reflector plane at 20 mm (Z 7.8, roughness alpha),
    wide receive cone so that the rough echo reaches many elements."""
    sc = scenes.Scene(np.array([[1.5, 0.0, 1540.0], [7.8, 0.0, 1540.0]]),
                      np.array([-20, -20, 0, 20, 20, 40.0]) * MM, 0, np.zeros((0, 9)), np.zeros((0, 2), np.int32),
                      np.zeros((0, 4)), np.zeros((0, 2), np.int32), np.array([[0.0, 0.0, 1.0, 20 * MM]]),
                      np.array([[1, 0]], np.int32), np.zeros((0, 4)), rough=np.array([0.0, alpha]))
    w = scenes.tiny(rays_per_element=rays_per_element)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(15.0), alpha_c=math.radians(45.0),
                              rough_direct_only=direct_only, max_bounces=1)
    return dataclasses.replace(w, scene=sc, acq=acq)


def _rough_floor_under_plane_workload(alpha, z_mid, direct_only, rays_per_element=512):
    """Water, then a smooth plane at 10 mm into a layer of impedance z_mid
    (1.5: matched, no bending and no loss; 1.6: mismatched), then the rough
    reflector plane at 20 mm (Z 7.8).  Every echo of the rough floor crosses
    the smooth plane on its way back, and up to three interactions are
    followed (down through the plane, the floor, up through the plane)."""
    mats = np.array([[1.5, 0.0, 1540.0], [z_mid, 0.0, 1540.0], [7.8, 0.0, 1540.0]])
    pln = np.array([[0.0, 0.0, 1.0, 10 * MM], [0.0, 0.0, 1.0, 20 * MM]])
    sc = scenes.Scene(mats, np.array([-20, -20, 0, 20, 20, 40.0]) * MM, 0, np.zeros((0, 9)),
                      np.zeros((0, 2), np.int32), np.zeros((0, 4)), np.zeros((0, 2), np.int32), pln,
                      np.array([[1, 0], [2, 1]], np.int32), np.zeros((0, 4)), rough=np.array([0.0, 0.0, alpha]))
    w = scenes.tiny(rays_per_element=rays_per_element)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(15.0), alpha_c=math.radians(45.0),
                              rough_direct_only=direct_only, max_bounces=3)
    return dataclasses.replace(w, scene=sc, acq=acq)


def _signal_by_element(oracle, make, parts=16):
    """Per-element received signal (summed over time) of `parts`
    independent replicas (different Philox keys) of both estimators."""
    sums = {}
    for direct_only in (1, 0):
        w = make(direct_only)
        ps = [oracle.trace(w, seed=0x5EED0001 + 7919 * k)[0].sum(2)[0] for k in range(parts)]
        sums[direct_only] = np.array(ps)
    return sums[1], sums[0]                       # [parts, E]


def _assert_same_expectation(a, b, parts=16):
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / parts + b.var(0, ddof=1) / parts)
    tot_a, tot_b = a.sum(1), b.sum(1)
    se_tot = math.sqrt(tot_a.var(ddof=1) / parts + tot_b.var(ddof=1) / parts)
    assert abs(tot_a.mean() - tot_b.mean()) < 5 * se_tot, (tot_a.mean(), tot_b.mean(), se_tot)
    bad = np.abs(ma - mb) > 5 * se + 1e-30
    assert bad.mean() < 0.05, (np.nonzero(bad)[0], ma[bad], mb[bad], se[bad])
    return tot_a, tot_b


@pytest.mark.parametrize("alpha", [0.3, 0.8])
def test_transducer_sampling_at_rough_boundaries_is_unbiased(oracle, alpha):
    """Per-element received signal (summed over time) with transducer
    sampling + balance heuristic equals the direct-hits-only signal within
    5 standard errors of their difference (16 independent ray subsets each)."""
    a, b = _signal_by_element(oracle, lambda direct_only: _rough_floor_workload(alpha, direct_only))
    tot_a, tot_b = _assert_same_expectation(a, b)
    # the secondary rays lower the variance of the total
    assert tot_b.std() < tot_a.std()


@pytest.mark.parametrize("z_mid", [1.5, 1.6])
def test_transducer_sampling_under_a_smooth_boundary_is_unbiased(oracle, z_mid):
    """A smooth plane between the rough floor and the array: the balanced
    estimator still equals the direct-hits-only one (a secondary ray that
    crosses a boundary records nothing, so the echo is not counted twice),
    and the totals agree within 5 standard errors, where double counting
    would give about twice the signal."""
    a, b = _signal_by_element(oracle, lambda direct_only: _rough_floor_under_plane_workload(0.5, z_mid,
                                                                                            direct_only))
    tot_a, tot_b = _assert_same_expectation(a, b)
    assert tot_a.mean() > 0 and abs(tot_b.mean() / tot_a.mean() - 1.0) < 0.2
    w = _rough_floor_under_plane_workload(0.5, z_mid, 0)
    _, st = oracle.trace(w)
    # every rough-boundary secondary ray that is cast crosses the plane
    assert st["nee_cast"] > 1000 and st["nee_blocked"] == st["nee_cast"]


def test_surface_records_in_the_event_log(oracle):
    """One ray onto the rough floor: a kind-5 record from the hit point at
    time t + 20 mm / c + r / c toward the drawn element, before the
    boundary's own event."""
    w = _rough_floor_workload(0.5, 0)
    rays = [dict(o=(0.0, 0.0, 0.0), d=(0.0, 0.0, 1.0), w=1.0, t=0.0, ray=r, elem=5) for r in range(200)]
    ev, st, _ = oracle.trace_rays(w, rays, cap=4000)
    surf = [e for e in ev if e["kind"] == "surface"]
    assert st["surface_events"] == 200 and len(surf) == st["nee_cast"] - st["nee_blocked"] > 20
    for e in surf:
        xe = (e["elem"] - 31.5) * w.acq.pitch
        r = math.hypot(xe, 20 * MM)
        assert e["t"] == pytest.approx(20 * MM / 1540.0 + r / 1540.0, rel=1e-12)
        assert np.allclose(e["pos"], (0.0, 0.0, 20 * MM), atol=1e-15)
        assert e["value"] > 0
