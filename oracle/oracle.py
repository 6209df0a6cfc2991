"""ctypes wrapper around the FP64 C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never does.  It imports
nothing from the HIP package.  Inputs are plain objects carrying numpy arrays
and scalars (the seeded workload generator's scene / acquisition / grid).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")


SAN_LIB_PATH = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so (portable -O2, no FMA contraction),
    or with sanitize into liboracle_san.so: AddressSanitizer and
    UndefinedBehaviorSanitizer, every report fatal, serial (no OpenMP).  A
    process that loads the sanitized library needs libasan preloaded."""
    out = SAN_LIB_PATH if sanitize else LIB_PATH
    opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
           if sanitize else ["-O2", "-fopenmp"])
    cmd = ["gcc", *opt, "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", os.path.join(HERE, "oracle.c"), "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class Acq(C.Structure):
    _fields_ = [("n_elements", C.c_int64), ("n_tx", C.c_int64), ("n_samples", C.c_int64),
                ("rays_per_element", C.c_int64), ("max_bounces", C.c_int64), ("binning", C.c_int64),
                ("pitch", C.c_double), ("elevation", C.c_double), ("f_c", C.c_double), ("f_s", C.c_double),
                ("c0", C.c_double), ("n_cycles", C.c_double), ("r_s", C.c_double), ("max_path", C.c_double),
                ("alpha_m", C.c_double), ("alpha_c", C.c_double), ("seed", C.c_uint64),
                ("angles", C.POINTER(C.c_double)), ("pdf", C.POINTER(C.c_float)),
                ("cdf", C.POINTER(C.c_float)), ("element_choice", C.c_int64), ("scheme", C.c_int64),
                ("radius", C.c_double), ("rough_direct_only", C.c_int64)]


class SceneS(C.Structure):
    _fields_ = [("n_mat", C.c_int64), ("n_tri", C.c_int64), ("n_sph", C.c_int64), ("n_pln", C.c_int64),
                ("n_scat", C.c_int64), ("top_medium", C.c_int64),
                ("mat", C.POINTER(C.c_double)), ("box", C.POINTER(C.c_double)),
                ("tri", C.POINTER(C.c_double)), ("tri_mat", C.POINTER(C.c_int32)),
                ("sph", C.POINTER(C.c_double)), ("sph_mat", C.POINTER(C.c_int32)),
                ("pln", C.POINTER(C.c_double)), ("pln_mat", C.POINTER(C.c_int32)),
                ("scat", C.POINTER(C.c_double)), ("rough", C.POINTER(C.c_double))]


STAT_FIELDS = ["rays", "segments", "reflect", "transmit", "tir", "scatter_events", "nee_zero", "nee_cast",
               "nee_blocked", "direct_hits", "records", "dropped", "edge_band", "term_box", "term_bounce",
               "term_time", "term_path", "media_mismatch", "term_rough", "surface_events", "surface_zero"]


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in STAT_FIELDS}


class Event(C.Structure):
    _fields_ = [("kind", C.c_int64), ("tx", C.c_int64), ("elem", C.c_int64), ("seg", C.c_int64),
                ("id", C.c_int64), ("t", C.c_double), ("value", C.c_double), ("x", C.c_double),
                ("y", C.c_double), ("z", C.c_double)]


class Ray(C.Structure):
    _fields_ = [("o", C.c_double * 3), ("d", C.c_double * 3), ("w", C.c_double), ("t", C.c_double),
                ("tx", C.c_int64), ("elem", C.c_int64), ("ray", C.c_int64), ("medium", C.c_int64)]


EVENT_KINDS = {0: "direct", 1: "scatter", 2: "reflect", 3: "transmit", 4: "end", 5: "surface"}

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", LIB_PATH)   # another build (e.g. the sanitized one)
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(path)
        P = C.POINTER
        L.or_trace.argtypes = [P(Acq), P(SceneS), C.c_int, P(C.c_double), P(Stats)]
        L.or_trace_subset.argtypes = [P(Acq), P(SceneS), C.c_int, C.c_int64, P(C.c_double), P(C.c_double),
                                      P(Stats)]
        L.or_trace_rays.argtypes = [P(Acq), P(SceneS), P(Ray), C.c_int64, P(Event), C.c_int64,
                                    P(C.c_int64), P(C.c_double), P(Stats)]
        grad_args = [P(C.c_double), C.c_int, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double),
                     P(C.c_double)]
        L.or_trace_grad.argtypes = [P(Acq), P(SceneS), C.c_int, C.c_int64] + grad_args
        L.or_trace_rays_grad.argtypes = [P(Acq), P(SceneS), P(Ray), C.c_int64] + grad_args
        L.or_trace_grad_edges.argtypes = [P(Acq), P(SceneS), C.c_int, C.c_int64, P(C.c_double), C.c_int,
                                          P(C.c_double), P(C.c_double)]
        L.or_edge_family.argtypes = [P(Acq), P(SceneS), P(C.c_double), C.c_int64, C.c_int64, C.c_int64, C.c_int,
                                     C.c_int64, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double),
                                     P(C.c_uint64), C.c_int, P(C.c_double)]
        L.or_pulse_taps.argtypes = [P(Acq), P(C.c_double), C.c_int64]
        L.or_pulse.argtypes = [P(Acq), C.c_int64, P(C.c_double), P(C.c_double)]
        L.or_das.argtypes = [P(Acq), C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double,
                             P(C.c_double), C.c_int, P(C.c_double)]
        L.or_das_points.argtypes = [P(Acq), P(C.c_double), C.c_int64, P(C.c_double), P(C.c_double)]
        L.or_envelope.argtypes = [C.c_int64, P(C.c_double), C.c_double, P(C.c_double), P(C.c_double)]
        L.or_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.or_hemisphere.argtypes = [C.c_double, C.c_double, P(C.c_double)]
        L.or_directivity.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_directivity.restype = C.c_double
        L.or_interface.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double, C.c_double,
                                   P(C.c_double), P(C.c_double)]
        L.or_synthesize.argtypes = [P(Acq), P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double)]
        L.or_interface_rough.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double, P(C.c_double), P(C.c_double),
                                         P(C.c_double)]
        L.or_onb.argtypes = [P(C.c_double), P(C.c_double), P(C.c_double)]
        L.or_ggx_sample.argtypes = [P(C.c_double), C.c_double, C.c_double, C.c_double, P(C.c_double)]
        L.or_ggx_d.argtypes = [C.c_double, C.c_double]
        L.or_ggx_d.restype = C.c_double
        L.or_ggx_g1.argtypes = [C.c_double, C.c_double]
        L.or_ggx_g1.restype = C.c_double
        L.or_delay.argtypes = [P(Acq), C.c_int64, C.c_int64]
        L.or_delay.restype = C.c_double
        L.or_closest_hit.argtypes = [P(SceneS), P(C.c_double), P(C.c_double), C.c_int64, P(C.c_double)]
        L.or_closest_hit.restype = C.c_int64
        L.or_crossings.argtypes = [P(SceneS), P(C.c_double), P(C.c_double), C.c_double, P(C.c_double),
                                   C.c_int64]
        L.or_crossings.restype = C.c_int64
        L.or_element_geometry.argtypes = [P(Acq), C.c_int64, P(C.c_double)]
        L.or_cone_elements.argtypes = [P(Acq), P(C.c_double), P(C.c_int64), P(C.c_int64)]
        L.or_rough_fcos.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double, C.c_double,
                                    P(C.c_double), P(C.c_double)]
        L.or_rough_fcos.restype = C.c_double
        L.or_sector_points.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                                       C.c_double, P(C.c_double)]
        L.or_scan_convert.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                                      C.c_double, P(C.c_double), C.c_int64, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, P(C.c_double)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class _Keep:
    """Holds numpy buffers alive while a ctypes struct points at them."""

    def __init__(self):
        self.bufs = []

    def f64(self, x, n=None):
        a = np.ascontiguousarray(np.asarray(x, np.float64))
        if n is not None:
            a = a.reshape(-1, n)
        self.bufs.append(a)
        return a

    def i32(self, x):
        a = np.ascontiguousarray(np.asarray(x, np.int32).reshape(-1, 2))
        self.bufs.append(a)
        return a

    def f32(self, x):
        a = np.ascontiguousarray(np.asarray(x, np.float32))
        self.bufs.append(a)
        return a


def make_acq(acq, seed, keep, pdf=None, cdf=None):
    ang = keep.f64(acq.angles)
    s = Acq(n_elements=acq.n_elements, n_tx=len(ang), n_samples=acq.n_samples,
            rays_per_element=acq.rays_per_element, max_bounces=acq.max_bounces, binning=acq.binning,
            pitch=acq.pitch, elevation=acq.elevation, f_c=acq.f_c, f_s=acq.f_s, c0=acq.c0,
            n_cycles=acq.n_cycles, r_s=acq.r_s, max_path=acq.max_path, alpha_m=acq.alpha_m,
            alpha_c=acq.alpha_c, seed=int(seed) & 0xFFFFFFFFFFFFFFFF, angles=_dp(ang),
            element_choice=int(getattr(acq, "element_choice", 0)), scheme=int(getattr(acq, "scheme", 0)),
            radius=float(getattr(acq, "radius", 0.0)),
            rough_direct_only=int(getattr(acq, "rough_direct_only", 0)))
    if pdf is not None:
        s.pdf = _fp(keep.f32(pdf))
        s.cdf = _fp(keep.f32(cdf))
    return s


def make_scene(sc, keep):
    mat = keep.f64(sc.materials, 3)
    box = keep.f64(sc.box)
    tri = keep.f64(sc.tri, 9)
    sph = keep.f64(sc.sph, 4)
    pln = keep.f64(sc.pln, 4)
    scat = keep.f64(sc.scat, 4)
    rough = getattr(sc, "rough", None)
    s = SceneS(n_mat=len(mat), n_tri=len(tri), n_sph=len(sph), n_pln=len(pln), n_scat=len(scat),
               top_medium=int(sc.top_medium), mat=_dp(mat), box=_dp(box), tri=_dp(tri),
               tri_mat=_ip(keep.i32(sc.tri_mat)), sph=_dp(sph), sph_mat=_ip(keep.i32(sc.sph_mat)),
               pln=_dp(pln), pln_mat=_ip(keep.i32(sc.pln_mat)), scat=_dp(scat))
    if rough is not None:
        s.rough = _dp(keep.f64(rough))
    return s


def trace(workload, n_threads: int = 0, ray_stride: int = 1, seed=None, pdf=None, cdf=None, rec_hist=False):
    """Channel data ch_raw[tx][e][n] (float64) and trace statistics; with
    rec_hist also the |c| histogram [tx][e_emit][1024] of the contributions."""
    keep = _Keep()
    acq = workload.acq
    a = make_acq(acq, workload.seed if seed is None else seed, keep, pdf, cdf)
    s = make_scene(workload.scene, keep)
    out = np.zeros((acq.n_tx, acq.n_elements, acq.n_samples), np.float64)
    rh = np.zeros((acq.n_tx, acq.n_elements, 1024), np.float64) if rec_hist else None
    st = Stats()
    rc = lib().or_trace_subset(C.byref(a), C.byref(s), int(n_threads), int(ray_stride), _dp(out),
                               _dp(rh) if rec_hist else None, C.byref(st))
    if rc != 0:
        raise RuntimeError(f"or_trace failed ({rc})")
    if rec_hist:
        return out, st.as_dict(), rh
    return out, st.as_dict()


def trace_rays(workload, rays, cap=4096, seed=None, with_hist=False):
    """Trace explicit rays; returns (events list of dicts, stats, optional ch_raw)."""
    keep = _Keep()
    acq = workload.acq
    a = make_acq(acq, workload.seed if seed is None else seed, keep)
    s = make_scene(workload.scene, keep)
    arr = (Ray * len(rays))()
    for i, r in enumerate(rays):
        arr[i].o[:] = list(map(float, r["o"]))
        arr[i].d[:] = list(map(float, r["d"]))
        arr[i].w = float(r.get("w", 1.0))
        arr[i].t = float(r.get("t", 0.0))
        arr[i].tx = int(r.get("tx", 0))
        arr[i].elem = int(r.get("elem", 0))
        arr[i].ray = int(r.get("ray", 0))
        arr[i].medium = int(r.get("medium", workload.scene.top_medium))
    ev = (Event * cap)()
    n_ev = C.c_int64(0)
    st = Stats()
    hist = np.zeros((acq.n_tx, acq.n_elements, acq.n_samples)) if with_hist else None
    rc = lib().or_trace_rays(C.byref(a), C.byref(s), arr, len(rays), ev, cap, C.byref(n_ev),
                             _dp(hist) if with_hist else None, C.byref(st))
    if rc != 0:
        raise RuntimeError(f"or_trace_rays failed ({rc})")
    events = [dict(kind=EVENT_KINDS[ev[i].kind], tx=ev[i].tx, elem=ev[i].elem, seg=ev[i].seg, id=ev[i].id,
                   t=ev[i].t, value=ev[i].value, pos=(ev[i].x, ev[i].y, ev[i].z))
              for i in range(min(n_ev.value, cap))]
    return events, st.as_dict(), hist


def _ray_array(workload, rays):
    arr = (Ray * max(1, len(rays)))()
    for i, r in enumerate(rays):
        arr[i].o[:] = list(map(float, r["o"]))
        arr[i].d[:] = list(map(float, r["d"]))
        arr[i].w = float(r.get("w", 1.0))
        arr[i].t = float(r.get("t", 0.0))
        arr[i].tx = int(r.get("tx", 0))
        arr[i].elem = int(r.get("elem", 0))
        arr[i].ray = int(r.get("ray", 0))
        arr[i].medium = int(r.get("medium", workload.scene.top_medium))
    return arr


def trace_grad(workload, g, attach_choice=False, ray_stride=1, n_threads=0, seed=None, rays=None):
    """Forward-mode gradient of J = sum g(t) c over the records of the same
    paths as trace(..., ray_stride) (or of explicit `rays`): returns
    dict(J, z [n_mat], alpha [n_mat], sph [n_sph][3], amp [n_scat])."""
    keep = _Keep()
    acq, sc = workload.acq, workload.scene
    a = make_acq(acq, workload.seed if seed is None else seed, keep)
    s = make_scene(sc, keep)
    gg = keep.f64(np.ascontiguousarray(g, np.float64).reshape(acq.n_tx, acq.n_elements, acq.n_samples))
    nm, ns, nk = len(sc.materials), len(sc.sph), len(sc.scat)
    J = C.c_double()
    gz, ga, gs, gk = np.zeros(nm), np.zeros(nm), np.zeros((ns, 3)), np.zeros(max(nk, 1))
    tail = [_dp(gg), int(bool(attach_choice)), C.byref(J), _dp(gz), _dp(ga), _dp(gs), _dp(gk)]
    if rays is None:
        rc = lib().or_trace_grad(C.byref(a), C.byref(s), int(n_threads), int(ray_stride), *tail)
    else:
        arr = _ray_array(workload, rays)
        rc = lib().or_trace_rays_grad(C.byref(a), C.byref(s), arr, len(rays), *tail)
    if rc != 0:
        raise RuntimeError(f"or_trace_grad failed ({rc})")
    return dict(J=J.value, z=gz, alpha=ga, sph=gs, amp=gk[:nk])


def trace_grad_edges(workload, g, ray_stride=1, n_scan=16, n_threads=0, seed=None):
    """Element-edge terms of the direct hits (element edges, aperture ends,
    elevation edges) that trace_grad's interior derivative leaves out,
    integrated exactly along the emission origin's lateral coordinate (choice
    attached): dict(z [n_mat], sph [n_sph][3]).  trace_grad(...,
    attach_choice=True) plus these estimates the derivative of the expected
    data where direct hits carry the only discontinuities."""
    keep = _Keep()
    acq, sc = workload.acq, workload.scene
    a = make_acq(acq, workload.seed if seed is None else seed, keep)
    s = make_scene(sc, keep)
    gg = keep.f64(np.ascontiguousarray(g, np.float64).reshape(acq.n_tx, acq.n_elements, acq.n_samples))
    nm, ns = len(sc.materials), len(sc.sph)
    cz, cs = np.zeros(nm), np.zeros((max(ns, 1), 3))
    rc = lib().or_trace_grad_edges(C.byref(a), C.byref(s), int(n_threads), int(ray_stride), _dp(gg), int(n_scan),
                                   _dp(cz), _dp(cs))
    if rc != 0:
        raise RuntimeError(f"or_trace_grad_edges failed ({rc})")
    return dict(z=cz, sph=cs[:ns])


def edge_family(workload, g, tx, e, ray, u0, attach=False, n_scan=16, seed=None):
    """One path family of trace_grad_edges at the origin coordinates u0:
    dict(F [n], dF [n][n_mat + 3 n_sph], X [n][2], sig [n], B [n_mat + 3 n_sph])
    (see or_edge_family)."""
    keep = _Keep()
    acq, sc = workload.acq, workload.scene
    a = make_acq(acq, workload.seed if seed is None else seed, keep)
    s = make_scene(sc, keep)
    gg = keep.f64(np.ascontiguousarray(g, np.float64).reshape(acq.n_tx, acq.n_elements, acq.n_samples))
    np_ = len(sc.materials) + 3 * len(sc.sph)
    uu = np.ascontiguousarray(u0, np.float64)
    n = len(uu)
    F, dF, X = np.zeros(n), np.zeros((n, np_)), np.zeros((n, 2))
    sig, B = np.zeros(n, np.uint64), np.zeros(max(np_, 1))
    rc = lib().or_edge_family(C.byref(a), C.byref(s), _dp(gg), int(tx), int(e), int(ray), int(bool(attach)), n,
                              _dp(uu), _dp(F), _dp(dF), _dp(X), sig.ctypes.data_as(C.POINTER(C.c_uint64)),
                              int(n_scan), _dp(B))
    if rc != 0:
        raise RuntimeError(f"or_edge_family failed ({rc})")
    return dict(F=F, dF=dF, X=X, sig=sig, B=B[:np_])


def pulse_taps(acq):
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    K = lib().or_pulse_taps(C.byref(a), None, 0)
    taps = np.zeros((2 * K + 1, 2))
    lib().or_pulse_taps(C.byref(a), _dp(taps), 2 * K + 1)
    return K, taps[:, 0] + 1j * taps[:, 1]


def pulse(acq, ch_raw):
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    x = np.ascontiguousarray(ch_raw, np.float64)
    if x.shape[-1] != acq.n_samples:
        raise ValueError("last axis must hold n_samples samples")
    y = np.zeros(x.shape + (2,), np.float64)
    if lib().or_pulse(C.byref(a), x.size // acq.n_samples, _dp(x), _dp(y)) != 0:
        raise RuntimeError("or_pulse failed")
    return y[..., 0] + 1j * y[..., 1]


def _rf_pairs(ch_rf, acq=None):
    z = np.asarray(ch_rf)
    if np.iscomplexobj(z):
        z = np.stack([z.real, z.imag], -1)
    if acq is not None and z.shape != (len(acq.angles), acq.n_elements, acq.n_samples, 2):
        raise ValueError(f"channel data shape {z.shape[:-1]} does not match the acquisition")
    return np.ascontiguousarray(z, np.float64)


def das(acq, grid, ch_rf, n_threads: int = 0):
    """Compounded IQ image [nx][nz] (complex128)."""
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    rf = _rf_pairs(ch_rf, acq)
    iq = np.zeros((grid.nx, grid.nz, 2))
    rc = lib().or_das(C.byref(a), grid.nx, grid.nz, grid.x0, grid.x1, grid.z0, grid.z1, _dp(rf),
                      int(n_threads), _dp(iq))
    if rc != 0:
        raise RuntimeError("or_das failed")
    return iq[..., 0] + 1j * iq[..., 1]


def das_points(acq, xz, ch_rf):
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    rf = _rf_pairs(ch_rf, acq)
    pts = np.ascontiguousarray(np.asarray(xz, np.float64).reshape(-1, 2))
    iq = np.zeros((len(pts), 2))
    if lib().or_das_points(C.byref(a), _dp(pts), len(pts), _dp(rf), _dp(iq)) != 0:
        raise RuntimeError("or_das_points failed")
    return iq[:, 0] + 1j * iq[:, 1]


def envelope(iq, dr_db=90.0):
    z = np.ascontiguousarray(np.stack([np.real(iq), np.imag(iq)], -1), np.float64)
    n = z.size // 2
    env = np.zeros(n)
    bm = np.zeros(n)
    lib().or_envelope(n, _dp(z), float(dr_db), _dp(env), _dp(bm))
    shape = np.shape(iq)
    return env.reshape(shape), bm.reshape(shape)


# ---------------------------------------------------------------- building blocks
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    lib().or_philox(c, k, out)
    return [int(v) for v in out]


def hemisphere(a, b):
    d = (C.c_double * 3)()
    lib().or_hemisphere(float(a), float(b), d)
    return np.array(d[:])


def directivity(alpha, alpha_m, alpha_c):
    return lib().or_directivity(float(alpha), float(alpha_m), float(alpha_c))


def interface(d, n, z_front, z_back, y):
    dd = (C.c_double * 3)(*map(float, d))
    nn = (C.c_double * 3)(*map(float, n))
    out = (C.c_double * 3)()
    R = C.c_double(0)
    refl = lib().or_interface(dd, nn, float(z_front), float(z_back), float(y), out, C.byref(R))
    return bool(refl), np.array(out[:]), R.value


def synthesize(acq, ch_sa, angles):
    """Plane-wave channel data [n_ang][E][S] synthesised from synthetic-aperture
    data [E][E][S] (float64)."""
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    x = np.ascontiguousarray(np.asarray(ch_sa, np.float64))
    ang = np.ascontiguousarray(np.asarray(angles, np.float64))
    out = np.zeros((len(ang), acq.n_elements, acq.n_samples))
    rc = lib().or_synthesize(C.byref(a), _dp(x), _dp(ang), len(ang), _dp(out))
    assert rc == 0
    return out


def interface_rough(d, n, z_front, z_back, alpha, y, xi1, xi2):
    """(kind, new direction, A_r^2, weight factor); kind 1 reflect, 0 transmit, -1 absorbed."""
    dd = (C.c_double * 3)(*map(float, d))
    nn = (C.c_double * 3)(*map(float, n))
    out = (C.c_double * 3)()
    R, wf = C.c_double(0), C.c_double(0)
    k = lib().or_interface_rough(dd, nn, float(z_front), float(z_back), float(alpha), float(y), float(xi1),
                                 float(xi2), out, C.byref(R), C.byref(wf))
    return int(k), np.array(out[:]), R.value, wf.value


def onb(n):
    nn = (C.c_double * 3)(*map(float, n))
    t, b = (C.c_double * 3)(), (C.c_double * 3)()
    lib().or_onb(nn, t, b)
    return np.array(t[:]), np.array(b[:])


def ggx_sample(n, alpha, xi1, xi2):
    nn = (C.c_double * 3)(*map(float, n))
    h = (C.c_double * 3)()
    lib().or_ggx_sample(nn, float(alpha), float(xi1), float(xi2), h)
    return np.array(h[:])


def ggx_d(alpha, cos_h):
    return lib().or_ggx_d(float(alpha), float(cos_h))


def ggx_g1(alpha, cos_v):
    return lib().or_ggx_g1(float(alpha), float(cos_v))


def delay(acq, tx, e):
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    return lib().or_delay(C.byref(a), int(tx), int(e))


def closest_hit(scene, o, d, skip=-1):
    keep = _Keep()
    s = make_scene(scene, keep)
    oo = (C.c_double * 3)(*map(float, o))
    dd = (C.c_double * 3)(*map(float, d))
    t = C.c_double(0)
    pid = lib().or_closest_hit(C.byref(s), oo, dd, int(skip), C.byref(t))
    return int(pid), t.value


def crossings(scene, o, d, t_max, cap=256):
    keep = _Keep()
    s = make_scene(scene, keep)
    oo = (C.c_double * 3)(*map(float, o))
    dd = (C.c_double * 3)(*map(float, d))
    ts = np.zeros(cap)
    n = lib().or_crossings(C.byref(s), oo, dd, float(t_max), _dp(ts), cap)
    return np.sort(ts[:min(n, cap)])


def element_geometry(acq):
    """(E, 4) array: element centre x, z and sin, cos of its normal's angle."""
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    out = np.zeros((acq.n_elements, 4))
    for e in range(acq.n_elements):
        lib().or_element_geometry(C.byref(a), e, _dp(out[e]))
    return out


def sector_points(radius, grid):
    """(nx*nz, 2) pixel positions of a sector grid (x0, x1 angles; z0, z1 depths)."""
    xz = np.zeros((grid.nx * grid.nz, 2))
    if lib().or_sector_points(float(radius), grid.nx, grid.nz, grid.x0, grid.x1, grid.z0, grid.z1, _dp(xz)) != 0:
        raise RuntimeError("or_sector_points failed")
    return xz


def scan_convert(radius, sector, img, cart, fill):
    """Bilinear scan conversion of img[nx][nz] on the sector grid onto the Cartesian grid."""
    src = np.ascontiguousarray(np.asarray(img, np.float64).reshape(sector.nx, sector.nz))
    out = np.zeros((cart.nx, cart.nz))
    rc = lib().or_scan_convert(float(radius), sector.nx, sector.nz, sector.x0, sector.x1, sector.z0, sector.z1,
                               _dp(src), cart.nx, cart.nz, cart.x0, cart.x1, cart.z0, cart.z1, float(fill), _dp(out))
    if rc != 0:
        raise RuntimeError("or_scan_convert failed")
    return out


def cone_elements(acq, q):
    """(e_lo, n_e) of the cone-restricted element choice at point q, or None."""
    keep = _Keep()
    a = make_acq(acq, 0, keep)
    qq = (C.c_double * 3)(*map(float, q))
    lo, n = C.c_int64(0), C.c_int64(0)
    ok = lib().or_cone_elements(C.byref(a), qq, C.byref(lo), C.byref(n))
    return (lo.value, n.value) if ok else None


def rough_fcos(wi, n, z1, z2, alpha, o):
    """(f(wi, o) |n.o|, density of o) of a rough boundary's sampler."""
    a = (C.c_double * 3)(*map(float, wi))
    b = (C.c_double * 3)(*map(float, n))
    c = (C.c_double * 3)(*map(float, o))
    pdf = C.c_double(0)
    v = lib().or_rough_fcos(a, b, float(z1), float(z2), float(alpha), c, C.byref(pdf))
    return v, pdf.value
