"""Host-only checks of the HIP library's BVH builder (no GPU needed).

The builder source is compiled with the host compiler into a small checker
that verifies the threaded layout (skip indices, leaf ranges, every
primitive exactly once, containment) and that the FP32 culling walk reaches
every primitive a brute-force FP64 test accepts.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2501_05828_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_05828_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    d = tmp_path_factory.mktemp("bvh")
    exe = str(d / "bvh_selfcheck")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "cpu", "bvh_selfcheck.cpp"),
                    os.path.join(CSRC, "bvh.cpp"), "-o", exe], check=True)
    return exe, d


def _run(checker, arr, kind, dilate, radius, n_rays, seed=1, leaf_max=None):
    exe, d = checker
    path = str(d / f"{kind}.bin")
    np.ascontiguousarray(arr, np.float64).tofile(path)
    extra = [str(leaf_max)] if leaf_max is not None else []
    r = subprocess.run([exe, path, str(len(arr)), kind, repr(dilate), repr(radius), str(n_rays), str(seed)] + extra,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.parametrize("leaf_max", [1, 4])
def test_triangle_bvh_bone_mesh(checker, leaf_max):
    """The library's single-triangle leaves, and leaves of up to four."""
    w = scenes.bone(rays_per_element=1)
    out = _run(checker, w.scene.tri, "tri", 1e-6, 0.0, 300, leaf_max=leaf_max)
    assert "missed 0" in out


def test_scatterer_bvh(checker):
    w = scenes.bone(rays_per_element=1, n_scatterers=20000)
    rs = w.acq.r_s
    out = _run(checker, w.scene.scat, "pt", rs * 1e-5 + 1e-6, rs, 300)
    assert "missed 0" in out


def test_small_and_degenerate_sets(checker):
    rng = np.random.default_rng(3)
    tri = rng.uniform(-0.01, 0.01, size=(5, 9))
    _run(checker, tri, "tri", 1e-6, 0.0, 200)
    pts = np.zeros((40, 4))                     # coincident points force index splits
    pts[:, 3] = 1.0
    _run(checker, pts, "pt", 1e-6, 1.5e-4, 50)
    _run(checker, rng.uniform(-0.01, 0.01, size=(1, 4)), "pt", 1e-6, 1.5e-4, 50)


@pytest.fixture(scope="module")
def grid_checker(tmp_path_factory):
    d = tmp_path_factory.mktemp("grid")
    exe = str(d / "grid_selfcheck")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "cpu", "grid_selfcheck.cpp"),
                    os.path.join(CSRC, "scatter_grid.cpp"), "-o", exe], check=True)
    return exe, d


def _run_grid(grid_checker, scat, box, r_s, n_seg, seed=1, rx=None):
    exe, d = grid_checker
    sp, bp = str(d / "s.bin"), str(d / "b.bin")
    np.ascontiguousarray(scat, np.float64).tofile(sp)
    np.ascontiguousarray(box, np.float64).tofile(bp)
    extra = [repr(float(v)) for v in rx] if rx is not None else []
    r = subprocess.run([exe, sp, str(len(scat)), bp, repr(r_s), str(n_seg), str(seed)] + extra,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_scatter_grid_walk_finds_every_capture_once(grid_checker):
    """Bone-phantom scatterers with an enlarged capture radius (more events
    per segment): the DDA walk with interval ownership reports exactly the
    brute-force capture set for every segment."""
    w = scenes.bone(rays_per_element=1, n_scatterers=20000)
    out = _run_grid(grid_checker, w.scene.scat, w.scene.box, 2e-3, 400)
    assert "bad=0" in out
    out = _run_grid(grid_checker, w.scene.scat, w.scene.box, w.acq.r_s, 400, seed=2)
    assert "bad=0" in out


def test_scatter_grid_edge_cases(grid_checker):
    box = np.array([-0.01, -0.01, 0.0, 0.01, 0.01, 0.02])
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform(box[:3], box[3:], size=(300, 3)),
                          np.array([[0.0, 0.0, 0.005], [0.01, 0.01, 0.02], [-0.01, 0.0, 0.0]])])  # on cell/box faces
    scat = np.hstack([pts, np.ones((len(pts), 1))])
    out = _run_grid(grid_checker, scat, box, 1.5e-3, 600)
    assert "bad=0" in out
    out = _run_grid(grid_checker, scat[:1], box, 1.5e-4, 100)
    assert "bad=0" in out


def _field(out, name):
    return float(out.split(name + "=")[1].split()[0])


@pytest.mark.parametrize("alpha_c_deg,r_s", [(2.0, 1.54e-4), (2.0, 2e-3), (20.0, 1e-3), (89.0, 1e-3), (90.0, 1e-3)])
def test_scatter_grid_audibility_cull(grid_checker, alpha_c_deg, r_s):
    """Scatterers left out of the grid because no element hears them: every
    capture point of a left-out scatterer lies outside the acceptance cone of
    all 128 element centres, and the walk over the smaller grid, clipped to
    the wedge around the cones, finds every capture whose point some element
    hears exactly once and reports nothing that is not a capture."""
    w = scenes.bone(rays_per_element=1, n_scatterers=20000)
    xe = (np.arange(128) - 63.5) * w.acq.pitch
    rx = (xe[0], xe[-1], np.radians(alpha_c_deg))
    out = _run_grid(grid_checker, w.scene.scat, w.scene.box, r_s, 1500, seed=3, rx=rx)
    assert "bad=0" in out and "heard_culled=0" in out, out
    kept = _field(out, "kept")
    assert _field(out, "heard") > 0, out
    if alpha_c_deg >= 90.0:
        assert kept == 20000
    if alpha_c_deg == 2.0:
        assert kept < 0.25 * 20000 and _field(out, "culled_events") > 0, out


@pytest.mark.parametrize("alpha_c_deg,r_s", [(2.0, 1.54e-4), (2.0, 2e-3), (15.0, 1e-3), (90.0, 1e-3)])
def test_scatter_grid_audibility_cull_convex(grid_checker, alpha_c_deg, r_s):
    """The same guarantees for a 128-element convex array of radius 50 mm
    spanning 70 degrees (apexes on the arc, radial axes): no capture that an
    element centre's cone holds is lost, and the walk reports nothing else."""
    w = scenes.convex(rays_per_element=1, n_scatterers=20000)
    R, E = w.acq.radius, w.acq.n_elements
    half = 0.5 * (E - 1) * w.acq.pitch / R
    rx = (0.0, 0.0, np.radians(alpha_c_deg), R, -half, half)
    out = _run_grid(grid_checker, w.scene.scat, w.scene.box, r_s, 1500, seed=5, rx=rx)
    assert "bad=0" in out and "heard_culled=0" in out, out
    kept = _field(out, "kept")
    assert _field(out, "heard") > 0, out
    if alpha_c_deg >= 90.0:
        assert kept == 20000
    if alpha_c_deg == 2.0:
        assert kept < 0.25 * 20000 and _field(out, "culled_events") > 0, out


def test_scatter_grid_cells_sized_by_occupied_cells(grid_checker):
    """The convex workload's 200,000 scatterers at alpha_c = 2 degrees: the
    audible ones fill a thin curved slab, a small part of their bounding box,
    so cells sized by the mean density over the box hold about 12.7
    registrations where occupied.  The builder shrinks the cells until the
    occupied ones hold about two (at most 1.5 times that), and the walk still
    finds every heard capture exactly once."""
    w = scenes.convex(rays_per_element=1)
    R, E = w.acq.radius, w.acq.n_elements
    half = 0.5 * (E - 1) * w.acq.pitch / R
    rx = (0.0, 0.0, w.acq.alpha_c, R, -half, half)
    out = _run_grid(grid_checker, w.scene.scat, w.scene.box, w.acq.r_s, 200, seed=6, rx=rx)
    assert "bad=0" in out and "heard_culled=0" in out, out
    per_cell = _field(out, "items") / _field(out, "occupied")
    print(f"[grid] convex workload: {per_cell:.2f} registrations per occupied cell")
    assert per_cell <= 3.0, out
