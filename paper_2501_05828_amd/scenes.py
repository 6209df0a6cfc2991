"""Seeded synthetic workloads (scenes, probe, acquisition, image grid).

This module only *builds inputs*: geometry, material tables, scatterer
clouds and parameter values.  It contains none of the simulation method's
arithmetic (no delays, no physics, no sampling), so both the HIP library and
the CPU oracle can be fed from it without sharing any method code.

Units are SI (metres, seconds, m/s) except impedance Z in MRayl and
attenuation alpha in dB/(cm MHz).  Frame: x lateral, y elevation, z depth;
a linear transducer's face is the plane z = 0 and faces +z; a convex one's is
a cylinder about the y axis that touches z = 0 at its middle, with its centre
of curvature at (0, 0, -radius).

The phantoms stand in for the paper's CT-derived vertebra in water (Sec. 4):
the real mesh and acquisitions are not available, so procedural tubes with
seeded surface noise, layered soft tissue and point-scatterer clouds of the
stated sizes are used instead.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

MM = 1e-3

NEAREST = 0
LINEAR = 1


@dataclass
class Scene:
    materials: np.ndarray        # (M,3) float64: Z [MRayl], alpha [dB/(cm MHz)], c [m/s]
    box: np.ndarray              # (6,) float64: xmin, ymin, zmin, xmax, ymax, zmax [m]
    top_medium: int              # material touching the transducer face
    tri: np.ndarray              # (NT,9) float64: v0, v1, v2
    tri_mat: np.ndarray          # (NT,2) int32: material on the front / back side
    sph: np.ndarray              # (NS,4) float64: centre xyz, radius
    sph_mat: np.ndarray          # (NS,2) int32: outside / inside material
    pln: np.ndarray              # (NP,4) float64: unit normal n, offset d (n.x = d)
    pln_mat: np.ndarray          # (NP,2) int32: front (n side) / back material
    scat: np.ndarray             # (K,4) float64: position xyz, amplitude
    rough: np.ndarray = None     # (M,) float64: GGX roughness alpha (Eq. 12) per material; None: all smooth

    def counts(self) -> dict:
        return dict(materials=len(self.materials), triangles=len(self.tri),
                    spheres=len(self.sph), planes=len(self.pln),
                    scatterers=len(self.scat))


ELEMENT_UNIFORM, ELEMENT_CONE = 0, 1
SCHEME_PLANE_WAVE, SCHEME_SYNTHETIC = 0, 1


@dataclass
class Acquisition:
    n_elements: int
    pitch: float                 # m
    elevation: float             # m (element height along y)
    f_c: float                   # Hz
    f_s: float                   # Hz
    n_samples: int
    angles: np.ndarray           # (T,) steering angles [rad]
    rays_per_element: int        # rays per element per transmit
    max_bounces: int
    max_path: float              # m
    alpha_m: float               # main-beam angle [rad]
    alpha_c: float               # cutoff angle [rad]
    c0: float                    # beamforming / delay speed of sound [m/s]
    n_cycles: float              # pulse length in cycles
    r_s: float                   # scatterer capture radius [m]
    binning: int = NEAREST
    element_choice: int = 0      # transducer sampling: 0 uniform over all elements, 1 over those in the cone
    scheme: int = 0              # 0 steered plane waves; 1 synthetic aperture (transmit t = element t alone)
    radius: float = 0.0          # 0 linear array; > 0 convex array of this radius (pitch = arc length)
    rough_direct_only: int = 0   # 1: no transducer sampling at rough boundaries (direct hits only)

    @property
    def n_tx(self) -> int:
        return int(len(self.angles))

    @property
    def n_rays(self) -> int:
        return self.n_tx * self.n_elements * self.rays_per_element


@dataclass
class Grid:
    nx: int
    nz: int
    x0: float
    x1: float
    z0: float
    z1: float
    sector: bool = False         # x0, x1 angles [rad] and z0, z1 depths below a convex array's face


@dataclass
class Workload:
    name: str
    scene: Scene
    acq: Acquisition
    grid: Grid
    seed: int = 0x5EED0001       # Philox key for the tracer
    scene_seed: int = 1
    apod: str = "hann"
    extra: dict = field(default_factory=dict)

    def with_rays(self, rays_per_element: int) -> "Workload":
        acq = dataclasses.replace(self.acq, rays_per_element=int(rays_per_element))
        return dataclasses.replace(self, acq=acq)


def _empty_i2():
    return np.zeros((0, 2), np.int32)


def _f64(x, n):
    a = np.asarray(x, np.float64).reshape(-1, n)
    return np.ascontiguousarray(a)


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, np.int32).reshape(-1, 2))


def tube_mesh(rng, axis_x, axis_z, n_phi, n_y, y_half, r_mean, r_amp):
    """Open tube along y with radius r_mean + r_amp * n(phi, y).

    n is a normalised sum of three seeded sinusoids in (phi, y), so it stays in
    [-1, 1] and is periodic in phi.  Triangles are wound so that the geometric
    normal (v1-v0)x(v2-v0) points out of the tube.
    """
    m = rng.integers(2, 7, size=3)
    ky = rng.integers(1, 4, size=3) * (2 * np.pi / (2 * y_half))
    amp = rng.uniform(0.5, 1.0, size=3)
    ph = rng.uniform(0, 2 * np.pi, size=3)
    phi = np.arange(n_phi) * (2 * np.pi / n_phi)
    y = -y_half + np.arange(n_y + 1) * (2 * y_half / n_y)
    P, Y = np.meshgrid(phi, y, indexing="ij")            # (n_phi, n_y+1)
    noise = sum(amp[i] * np.sin(m[i] * P + ky[i] * Y + ph[i]) for i in range(3)) / amp.sum()
    r = r_mean + r_amp * noise
    V = np.stack([axis_x + r * np.cos(P), Y, axis_z + r * np.sin(P)], -1)
    i = np.arange(n_phi)[:, None]
    j = np.arange(n_y)[None, :]
    ip = (i + 1) % n_phi
    a = V[i, j]
    b = V[i, j + 1]
    c = V[ip, j]
    d = V[ip, j + 1]
    t1 = np.stack([a, b, c], -2)                           # (n_phi, n_y, 3, 3)
    t2 = np.stack([c, b, d], -2)
    tri = np.stack([t1, t2], 2).reshape(-1, 9)
    return np.ascontiguousarray(tri, np.float64)


def tiny(scene_seed: int = 1, rays_per_element: int = 1024, n_scatterers: int = 2000) -> Workload:
    """Plain tracer, tiny: 64 elements, one 0-degree plane wave, 40 mm cube.

    Planar reflector at 20 mm depth (Z 7.8), one 3 mm sphere (Z 3.0) whose
    centre is uniform in the box and rejected if it would cut the reflector,
    2000 uniform scatterers with N(0,1) amplitudes.
    """
    rng = np.random.default_rng(scene_seed)
    box = np.array([-20 * MM, -20 * MM, 0.0, 20 * MM, 20 * MM, 40 * MM])
    mats = np.array([[1.5, 0.5, 1540.0],     # 0: medium
                     [7.8, 0.5, 1540.0],     # 1: reflector half-space z > 20 mm
                     [3.0, 0.5, 1540.0]])    # 2: sphere
    r = 3 * MM
    while True:
        cen = rng.uniform(box[:3] + r, box[3:] - r)
        if abs(cen[2] - 20 * MM) >= r:
            break
    sph = np.array([[cen[0], cen[1], cen[2], r]])
    sph_mat = np.array([[0 if cen[2] < 20 * MM else 1, 2]])
    pln = np.array([[0.0, 0.0, 1.0, 20 * MM]])
    pln_mat = np.array([[1, 0]])
    pos = rng.uniform(box[:3], box[3:], size=(n_scatterers, 3))
    amp = rng.normal(0.0, 1.0, size=(n_scatterers, 1))
    scene = Scene(_f64(mats, 3), box, 0, np.zeros((0, 9)), _empty_i2(),
                  _f64(sph, 4), _i32(sph_mat), _f64(pln, 4), _i32(pln_mat),
                  _f64(np.hstack([pos, amp]), 4))
    acq = Acquisition(64, 0.3 * MM, 4 * MM, 5e6, 40e6, 2048, np.deg2rad([0.0]),
                      rays_per_element, 4, 0.2, np.deg2rad(2.0), np.deg2rad(2.0),
                      1540.0, 5.0, 1540.0 / (2 * 5e6))
    grid = Grid(128, 256, -9.6 * MM, 9.6 * MM, 1 * MM, 40 * MM)
    return Workload("tiny", scene, acq, grid, scene_seed=scene_seed)


def _layers(rng, box, z_first=(4, 10), z_gap=(4, 10)):
    z1 = rng.uniform(*z_first) * MM
    z2 = z1 + rng.uniform(*z_gap) * MM
    Z = rng.uniform(1.4, 1.7, size=3)
    c = rng.uniform(1450, 1600, size=3)
    mats = [[Z[i], 0.5, c[i]] for i in range(3)]
    pln = np.array([[0.0, 0.0, 1.0, z1], [0.0, 0.0, 1.0, z2]])
    pln_mat = np.array([[1, 0], [2, 1]])
    return mats, pln, pln_mat, (z1, z2)


def bone(scene_seed: int = 1, rays_per_element: int = 78125, angles_deg=None,
         n_phi: int = 300, n_y: int = 100, n_scatterers: int = 50_000,
         grid_n=(512, 512)) -> Workload:
    """Plain tracer, bone phantom: 128 elements, 11 plane waves -10..10 deg.

    Three seeded soft-tissue slabs (Z in 1.4-1.7, c in 1450-1600), a 60k
    triangle tube (radius 8 mm +- 2 mm of sinusoidal noise, Z 7.8, 10
    dB/cm/MHz) and 50k scatterers with lognormal amplitudes (sigma 0.5).
    """
    rng = np.random.default_rng(scene_seed)
    if angles_deg is None:
        angles_deg = np.arange(-10, 11, 2)
    box = np.array([-30 * MM, -20 * MM, 0.0, 30 * MM, 20 * MM, 80 * MM])
    mats, pln, pln_mat, _ = _layers(rng, box)
    mats.append([7.8, 10.0, 1540.0])        # 3: bone
    ax = rng.uniform(-5, 5) * MM
    az = rng.uniform(35, 45) * MM
    tri = tube_mesh(rng, ax, az, n_phi, n_y, 25 * MM, 8 * MM, 2 * MM)
    tri_mat = np.tile(np.array([[2, 3]], np.int32), (len(tri), 1))
    pos = rng.uniform(box[:3], box[3:], size=(n_scatterers, 3))
    amp = np.exp(0.5 * rng.normal(size=(n_scatterers, 1)))
    scene = Scene(_f64(mats, 3), box, 0, tri, _i32(tri_mat), np.zeros((0, 4)), _empty_i2(),
                  _f64(pln, 4), _i32(pln_mat), _f64(np.hstack([pos, amp]), 4))
    acq = Acquisition(128, 0.3 * MM, 4 * MM, 5e6, 40e6, 4096, np.deg2rad(np.asarray(angles_deg, float)),
                      rays_per_element, 8, 0.2, np.deg2rad(2.0), np.deg2rad(2.0),
                      1540.0, 5.0, 1540.0 / (2 * 5e6))
    grid = Grid(grid_n[0], grid_n[1], -19.2 * MM, 19.2 * MM, 1 * MM, 79 * MM)
    w = Workload("bone", scene, acq, grid, scene_seed=scene_seed)
    w.extra.update(tube_axis=(ax, az))
    return w


def batched(scene_seed: int = 1, rays_per_element: int = 156250) -> Workload:
    """Bone phantom with 21 plane waves -20..20 deg, 2e7 rays per transmit,
    beamformed to a 1024x1024 compounded image with Hann apodisation."""
    w = bone(scene_seed, rays_per_element, angles_deg=np.arange(-20, 21, 2), grid_n=(1024, 1024))
    w.name = "batched"
    return w


def learned(scene_seed: int = 1, rays_per_element: int = 78125) -> Workload:
    """Bone phantom used to train and evaluate the learned emission proposal."""
    w = bone(scene_seed, rays_per_element)
    w.name = "learned"
    return w


def large(scene_seed: int = 1, rays_per_element: int = 124008, n_phi: int = 1000, n_y: int = 125,
          n_scatterers: int = 1_000_000) -> Workload:
    """Differentiable large scene: 192 elements, 21 angles, two 250k-triangle
    tubes, 4 spheres, 1e6 scatterers, six (Z, alpha) materials, linear
    (tent) binning so the channel data is continuous in arrival time."""
    rng = np.random.default_rng(scene_seed)
    box = np.array([-40 * MM, -20 * MM, 0.0, 40 * MM, 20 * MM, 80 * MM])
    mats, pln, pln_mat, (z1, z2) = _layers(rng, box)
    mats.append([7.8, 10.0, 1540.0])        # 3: bone
    mats.append([2.0, 1.0, 1540.0])         # 4: sphere material A
    mats.append([1.2, 0.3, 1540.0])         # 5: sphere material B
    axes = [(rng.uniform(-22, -12) * MM, rng.uniform(35, 45) * MM),
            (rng.uniform(12, 22) * MM, rng.uniform(45, 55) * MM)]
    tris = [tube_mesh(rng, a[0], a[1], n_phi, n_y, 25 * MM, 8 * MM, 2 * MM) for a in axes]
    tri = np.concatenate(tris, 0)
    tri_mat = np.tile(np.array([[2, 3]], np.int32), (len(tri), 1))
    sph = []
    while len(sph) < 4:
        r = rng.uniform(2, 4) * MM
        c = rng.uniform(box[:3] + r + 1 * MM, box[3:] - r - 1 * MM)
        if c[2] - r < z2 + 1 * MM:
            continue
        if any(np.hypot(c[0] - a[0], c[2] - a[1]) < 10 * MM + r + 1 * MM for a in axes):
            continue
        if any(np.linalg.norm(c - s[:3]) < r + s[3] + 1 * MM for s in sph):
            continue
        sph.append(np.array([c[0], c[1], c[2], r]))
    sph = np.array(sph)
    sph_mat = np.array([[2, 4], [2, 4], [2, 5], [2, 5]])
    pos = rng.uniform(box[:3], box[3:], size=(n_scatterers, 3))
    amp = np.exp(0.5 * rng.normal(size=(n_scatterers, 1)))
    scene = Scene(_f64(mats, 3), box, 0, tri, _i32(tri_mat), _f64(sph, 4), _i32(sph_mat),
                  _f64(pln, 4), _i32(pln_mat), _f64(np.hstack([pos, amp]), 4))
    acq = Acquisition(192, 0.3 * MM, 4 * MM, 5e6, 40e6, 4096, np.deg2rad(np.arange(-20, 21, 2.0)),
                      rays_per_element, 8, 0.2, np.deg2rad(2.0), np.deg2rad(2.0),
                      1540.0, 5.0, 1540.0 / (2 * 5e6), binning=LINEAR)
    grid = Grid(512, 512, -28.8 * MM, 28.8 * MM, 1 * MM, 79 * MM)
    w = Workload("large", scene, acq, grid, scene_seed=scene_seed)
    w.extra.update(tube_axes=axes)
    return w


def proposal_init(seed: int = 7):
    """Seeded initial parameters of the 34-64-64-64-1024 proposal network:
    He-normal weights, zero biases, laid out W1, b1, W2, b2, W3, b3, W4, b4
    with W stored (inputs, outputs).  Also the 16x2 random Fourier matrix
    (standard normal).  Inputs shared by the library and the reference."""
    rng = np.random.default_rng(seed)
    shapes = [(34, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64, 1024), (1024,)]
    parts = [rng.normal(0.0, np.sqrt(2.0 / sh[0]), size=sh).ravel() if len(sh) == 2 else np.zeros(sh)
             for sh in shapes]
    rff = rng.normal(size=(16, 2))
    return np.concatenate(parts).astype(np.float32), rff.astype(np.float32)


def convex_probe(w: Workload, radius: float, margin: float = 1 * MM) -> Workload:
    """The same scene seen through a convex array of the given radius (same
    element count and pitch, the pitch now the arc length).  The box top is
    raised above the array's ends by `margin`, and the image grid becomes a
    sector grid spanning the array's angles and the box depth."""
    half = 0.5 * w.acq.n_elements * w.acq.pitch / radius
    box = np.array(w.scene.box, np.float64).copy()
    box[2] = -radius * (1.0 - np.cos(half)) - margin
    scene = dataclasses.replace(w.scene, box=box)
    acq = dataclasses.replace(w.acq, radius=float(radius))
    grid = Grid(w.grid.nx, w.grid.nz, -half, half, 1 * MM, float(w.scene.box[5]) - 1 * MM, sector=True)
    out = dataclasses.replace(w, name=w.name + "-convex", scene=scene, acq=acq, grid=grid, extra=dict(w.extra))
    r_max = radius + grid.z1
    out.extra["cart_grid"] = Grid(w.grid.nx, w.grid.nz, -r_max * np.sin(half), r_max * np.sin(half),
                                  float(box[2]), float(w.scene.box[5]))
    return out


def tiny_convex(scene_seed: int = 1, rays_per_element: int = 1024, n_scatterers: int = 2000) -> Workload:
    """The tiny scene through a 64-element convex array of radius 20 mm
    (55 degrees of arc), receive angles alpha_m = 4, alpha_c = 10 deg (wider
    than the paper's 2 deg so that a small case records direct hits off the
    flat reflector)."""
    w = convex_probe(tiny(scene_seed, rays_per_element, n_scatterers), 20 * MM)
    w.acq = dataclasses.replace(w.acq, alpha_m=np.deg2rad(4.0), alpha_c=np.deg2rad(10.0))
    w.name = "tiny_convex"
    return w


def convex(scene_seed: int = 1, rays_per_element: int = 100_000, n_phi: int = 300, n_y: int = 100,
           n_scatterers: int = 200_000, radius: float = 50 * MM) -> Workload:
    """The paper's acquisition settings (Sec. 4) on a synthetic phantom: a
    128-element convex array of radius 50 mm spanning 70 degrees, 25 plane
    waves over -30..30 deg, 5 MHz, 5 cycles, fs 50 MHz, 10 bounces, 20 cm
    maximum path, alpha_m = alpha_c = 2 deg, 1e5 rays per element
    (1.28e7 per transmit, 3.2e8 per frame).  The phantom is the bone scene's
    recipe (three seeded soft-tissue slabs, a 60k-triangle noisy tube at
    35-45 mm, lognormal scatterers at the same density) in a box wide enough
    for the sector: x +-85 mm, y +-20 mm, z from above the array's ends to
    100 mm.  Sector grid 256 angles x 512 depths (1-90 mm), scan converted to
    512 x 512."""
    rng = np.random.default_rng(scene_seed)
    E, opening = 128, np.deg2rad(70.0)
    pitch = radius * opening / E
    box = np.array([-85 * MM, -20 * MM, -radius * (1.0 - np.cos(0.5 * opening)) - 1 * MM, 85 * MM, 20 * MM, 100 * MM])
    mats, pln, pln_mat, _ = _layers(rng, box)
    mats.append([7.8, 10.0, 1540.0])        # 3: bone
    ax = rng.uniform(-5, 5) * MM
    az = rng.uniform(35, 45) * MM
    tri = tube_mesh(rng, ax, az, n_phi, n_y, 25 * MM, 8 * MM, 2 * MM)
    tri_mat = np.tile(np.array([[2, 3]], np.int32), (len(tri), 1))
    pos = rng.uniform(box[:3], box[3:], size=(n_scatterers, 3))
    amp = np.exp(0.5 * rng.normal(size=(n_scatterers, 1)))
    scene = Scene(_f64(mats, 3), box, 0, tri, _i32(tri_mat), np.zeros((0, 4)), _empty_i2(),
                  _f64(pln, 4), _i32(pln_mat), _f64(np.hstack([pos, amp]), 4))
    acq = Acquisition(E, pitch, 4 * MM, 5e6, 50e6, 6912, np.deg2rad(np.linspace(-30.0, 30.0, 25)),
                      rays_per_element, 10, 0.2, np.deg2rad(2.0), np.deg2rad(2.0),
                      1540.0, 5.0, 1540.0 / (2 * 5e6), radius=float(radius))
    half = 0.5 * opening
    grid = Grid(256, 512, -half, half, 1 * MM, 90 * MM, sector=True)
    w = Workload("convex", scene, acq, grid, scene_seed=scene_seed)
    r_max = radius + 90 * MM
    w.extra.update(tube_axis=(ax, az),
                   cart_grid=Grid(512, 512, -r_max * np.sin(half), r_max * np.sin(half), float(box[2]), 90 * MM))
    return w


def _rough_bone(w: Workload, name: str, alpha: float = 0.5) -> Workload:
    rough = np.zeros(len(w.scene.materials))
    rough[3] = alpha                        # the tube's bone material
    out = dataclasses.replace(w, name=name, scene=dataclasses.replace(w.scene, rough=rough))
    return out


def bone_rough(scene_seed: int = 1, rays_per_element: int = 78125) -> Workload:
    """The bone workload with the bone's GGX roughness 0.5, the value the
    paper settles on for its vertebra (Sec. 4); the soft-tissue boundaries
    stay smooth."""
    return _rough_bone(bone(scene_seed, rays_per_element), "bone_rough")


def paper(scene_seed: int = 1, rays_per_element: int = 100_000, n_scatterers: int = 200_000) -> Workload:
    """The convex workload (the paper's acquisition settings) with the bone's
    roughness 0.5 as well: the whole of the paper's simulation set-up on the
    synthetic phantom."""
    return _rough_bone(convex(scene_seed, rays_per_element, n_scatterers=n_scatterers), "paper")


CONFIGS = {"tiny": tiny, "bone": bone, "batched": batched, "learned": learned, "large": large,
           "tiny_convex": tiny_convex, "convex": convex, "bone_rough": bone_rough, "paper": paper}


def make(name: str, **kw) -> Workload:
    return CONFIGS[name](**kw)


def synthetic_aperture(w: Workload) -> Workload:
    """The same scene and probe acquired element by element: transmit t fires
    element t alone without delay (n_tx = n_elements; the angles are unused),
    its rays drawn as in transmit 0 of a plane-wave set."""
    acq = dataclasses.replace(w.acq, scheme=SCHEME_SYNTHETIC, angles=np.zeros(w.acq.n_elements))
    return dataclasses.replace(w, name=w.name + "-sa", acq=acq)
