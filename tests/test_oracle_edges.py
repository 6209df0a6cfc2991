"""Oracle: element-edge terms of the direct hits (or_trace_grad_edges).

A direct hit is binned into the element whose face holds its landing
point, so moving a sphere moves contributions across element edges, the
ends of the aperture and the elevation edges; the interior derivative
(or_trace_grad) leaves these jumps out.  or_trace_grad_edges integrates
them exactly along the emission origin's lateral coordinate u0 of every
path family (Leibniz rule on [0, 1]).  Pinned here:

* the edge replay against or_trace: over all families of a small scene
  without scatterers, the replayed value at each family's own sampled u0
  sums to J = sum g ch_raw of or_trace (the same paths by a different
  code path);
* the Leibniz term against plain numerical differentiation: for single
  families (choice frozen, one sequence of primitives over u0), the
  central difference of the midpoint-rule integral of F over u0 equals
  the interior derivative plus the edge term, where the edge term is a
  large part of the derivative.

Both for a linear array and for a convex one (20 mm radius), where the
origin moves along the arc, the direction turns with it, the landing
coordinate is the arc angle and every element receives against its own
normal.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2501_05828_amd import scenes


def _workload(rays):
    """The small scene with its sphere under the aperture, no scatterers,
    linear binning and wide receive angles (many direct hits)."""
    w = scenes.tiny(rays_per_element=rays)
    acq = dataclasses.replace(w.acq, alpha_m=math.radians(10), alpha_c=math.radians(45), binning=scenes.LINEAR,
                              angles=np.deg2rad([0.0]))
    sph = np.array([[1.0e-3, 0.5e-3, 12.0e-3, 3.0e-3]])
    sc = dataclasses.replace(w.scene, sph=sph, sph_mat=np.array([[0, 2]], np.int32), scat=np.zeros((0, 4)))
    return dataclasses.replace(w, acq=acq, scene=sc)


def _adjoint(acq, seed):
    """Smooth random adjoint of one sign per half of the aperture: a jump
    of g at the centre edge, as well as at every element edge."""
    from scipy.ndimage import gaussian_filter1d
    rng = np.random.default_rng(seed)
    g = gaussian_filter1d(rng.normal(size=(acq.n_tx, acq.n_elements, acq.n_samples)), 40.0, axis=2) * 10
    return np.abs(g) * np.where(np.arange(acq.n_elements) < acq.n_elements // 2, 1.0, -1.0)[None, :, None]


def _u0(O, w, tx, e, ray):
    """The origin coordinate the family's own path draws (first word of the
    emission draw, counter (ray, e | tx << 16, 0, 0))."""
    key = (w.seed & 0xFFFFFFFF, (w.seed >> 32) & 0xFFFFFFFF)
    x = O.philox((ray, e | (tx << 16), 0, 0), key)
    return (int(x[0]) + 0.5) / 4294967296.0


@pytest.mark.parametrize("convex", [False, True])
def test_edge_replay_matches_trace(oracle, convex):
    O = oracle
    w = _workload(16)
    if convex:
        w = scenes.convex_probe(w, 20e-3)
    A = w.acq
    g = _adjoint(A, 5)
    ch, _ = O.trace(w)
    J_trace = float((ch * g).sum())
    J = 0.0
    for e in range(A.n_elements):
        for ray in range(A.rays_per_element):
            r = O.edge_family(w, g, 0, e, ray, [_u0(O, w, 0, e, ray)], n_scan=1)
            J += float(r["F"][0])
    print(f"[edges] J from the edge replay {J:.12e}, from or_trace {J_trace:.12e}")
    assert J_trace != 0.0
    assert abs(J - J_trace) <= 1e-9 * abs(J_trace)


@pytest.mark.parametrize("convex,families", [(False, 4), (True, 2)])
def test_edge_term_matches_quadrature(oracle, convex, families):
    O = oracle
    w = _workload(1024)
    if convex:
        w = scenes.convex_probe(w, 20e-3)
    A = w.acq
    g = _adjoint(A, 5)
    nm = len(w.scene.materials)
    coord = nm + 0                      # the sphere centre's x
    u_coarse = (np.arange(64) + 0.5) / 64
    u = (np.arange(100_000) + 0.5) / 100_000
    h = 1e-6      # the crossings move across many quadrature points, the path stays linear
    checked, dominant = 0, 0
    for i in range(0, A.n_elements * A.rays_per_element, 37):
        e, ray = i // A.rays_per_element, i % A.rays_per_element
        r = O.edge_family(w, g, 0, e, ray, u_coarse, n_scan=16)
        if not np.any(r["F"] != 0.0) or not np.any(r["dF"][:, coord] != 0.0) or r["B"][coord] == 0.0:
            continue
        r = O.edge_family(w, g, 0, e, ray, u, n_scan=16)
        if len(set(r["sig"].tolist())) != 1:
            continue

        def integral(dx):
            sph = w.scene.sph.copy()
            sph[0, 0] += dx
            ww = dataclasses.replace(w, scene=dataclasses.replace(w.scene, sph=sph))
            return O.edge_family(ww, g, 0, e, ray, u, n_scan=1)["F"].mean()

        fd = (integral(h) - integral(-h)) / (2 * h)
        interior, edge = r["dF"][:, coord].mean(), r["B"][coord]
        print(f"[edges] family (e {e}, ray {ray}): difference {fd:+.6e}, interior {interior:+.6e} + edge "
              f"{edge:+.6e} = {interior + edge:+.6e}")
        assert abs(fd - (interior + edge)) <= 0.02 * abs(fd)
        dominant += abs(edge) > 0.3 * abs(fd)
        checked += 1
        if checked == families:
            break
    assert checked == families and dominant >= 1
