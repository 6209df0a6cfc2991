"""ctypes binding of libultraray.so (include/ultraray.h), names kept 1:1.

Argument marshalling only: every step of the simulation runs in the HIP
library.  PyTorch provides device memory and the current HIP stream.  If the
library has not been built this module raises at load time; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libultraray.so")

UR_BIN_NEAREST, UR_BIN_LINEAR = 0, 1
UR_APOD_NONE, UR_APOD_HANN = 0, 1

STATUS = {0: "UR_OK", -1: "UR_ERR_INVALID_ARG", -2: "UR_ERR_CALL_ORDER", -3: "UR_ERR_OOM", -4: "UR_ERR_HIP",
          -5: "UR_ERR_SCENE", -6: "UR_ERR_CAPACITY", -7: "UR_ERR_UNSUPPORTED"}

P = C.POINTER


class SceneDesc(C.Structure):
    _fields_ = [("n_mat", C.c_int64), ("n_tri", C.c_int64), ("n_sph", C.c_int64), ("n_pln", C.c_int64),
                ("n_scat", C.c_int64), ("top_medium", C.c_int64),
                ("mat", P(C.c_double)), ("box", P(C.c_double)), ("tri", P(C.c_double)), ("tri_mat", P(C.c_int32)),
                ("sph", P(C.c_double)), ("sph_mat", P(C.c_int32)), ("pln", P(C.c_double)),
                ("pln_mat", P(C.c_int32)), ("scat", P(C.c_double)), ("rough", P(C.c_double))]


class ProbeDesc(C.Structure):
    _fields_ = [("n_elements", C.c_int64), ("pitch", C.c_double), ("elevation", C.c_double), ("f_c", C.c_double),
                ("radius", C.c_double)]


class AcqDesc(C.Structure):
    _fields_ = [("n_tx", C.c_int64), ("n_samples", C.c_int64), ("rays_per_element", C.c_int64),
                ("max_bounces", C.c_int64), ("binning", C.c_int64), ("f_s", C.c_double), ("c0", C.c_double),
                ("n_cycles", C.c_double), ("r_s", C.c_double), ("max_path", C.c_double), ("alpha_m", C.c_double),
                ("alpha_c", C.c_double), ("angles", P(C.c_double)), ("element_choice", C.c_int64),
                ("scheme", C.c_int64), ("rough_direct_only", C.c_int64)]


def _grid_desc(grid, apod, dynamic_range_db):
    return GridDesc(nx=grid.nx, nz=grid.nz, apod=apod, x0=grid.x0, x1=grid.x1, z0=grid.z0, z1=grid.z1,
                    dynamic_range_db=dynamic_range_db, sector=1 if getattr(grid, "sector", False) else 0)


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int64), ("nz", C.c_int64), ("apod", C.c_int64), ("x0", C.c_double), ("x1", C.c_double),
                ("z0", C.c_double), ("z1", C.c_double), ("dynamic_range_db", C.c_double), ("sector", C.c_int64)]


STAT_FIELDS = ["rays", "segments", "reflect", "transmit", "tir", "scatter_events", "nee_zero", "nee_cast",
               "nee_blocked", "direct_hits", "records", "dropped", "edge_band", "term_box", "term_bounce",
               "term_time", "term_path", "media_mismatch", "tri_nodes", "tri_tests", "scat_cells", "scat_tests",
               "shadow_nodes", "shadow_tri_tests", "term_rough", "surface_events", "surface_zero"]


class TraceStats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in STAT_FIELDS] + [("kernel_ms", C.c_double)]

    def as_dict(self):
        d = {f: int(getattr(self, f)) for f in STAT_FIELDS}
        d["kernel_ms"] = float(self.kernel_ms)
        return d


class Event(C.Structure):
    _fields_ = [("kind", C.c_int64), ("tx", C.c_int64), ("elem", C.c_int64), ("seg", C.c_int64), ("id", C.c_int64),
                ("t", C.c_double), ("value", C.c_double), ("x", C.c_double), ("y", C.c_double), ("z", C.c_double)]


class Ray(C.Structure):
    _fields_ = [("o", C.c_double * 3), ("d", C.c_double * 3), ("w", C.c_double), ("t", C.c_double),
                ("tx", C.c_int64), ("elem", C.c_int64), ("ray", C.c_int64), ("medium", C.c_int64)]


class GradDesc(C.Structure):
    _fields_ = [("amp", C.c_void_p), ("alpha", C.c_void_p), ("Z", C.c_void_p), ("sph_center", C.c_void_p),
                ("value", C.c_void_p), ("frozen_choice", C.c_int32), ("record_paths", C.c_int64)]


EVENT_KINDS = {0: "direct", 1: "scatter", 2: "reflect", 3: "transmit", 4: "end", 5: "surface"}

# (name, restype, argtypes) for every entry point declared in include/ultraray.h
_CTX = C.c_void_p
SIGNATURES = [
    ("ur_version", C.c_char_p, []),
    ("ur_context_create", C.c_int, [C.c_int, P(C.c_void_p)]),
    ("ur_context_destroy", None, [_CTX]),
    ("ur_last_error", C.c_char_p, [_CTX]),
    ("ur_scene_upload", C.c_int, [_CTX, P(SceneDesc)]),
    ("ur_transmit_setup", C.c_int, [_CTX, P(ProbeDesc), P(AcqDesc)]),
    ("ur_set_proposal", C.c_int, [_CTX, C.c_void_p, C.c_void_p]),
    ("ur_synthesize", C.c_int, [_CTX, C.c_void_p, P(C.c_double), C.c_int64, C.c_void_p, C.c_void_p]),
    ("ur_scan_convert", C.c_int, [_CTX, P(GridDesc), C.c_void_p, P(GridDesc), C.c_float, C.c_void_p, C.c_void_p]),
    ("ur_trace", C.c_int, [_CTX, C.c_uint64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, P(TraceStats),
                           C.c_void_p]),
    ("ur_set_limits", C.c_int, [_CTX, C.c_int64, C.c_int64]),
    ("ur_set_segment_queue", C.c_int, [_CTX, C.c_int64]),
    ("ur_pulse", C.c_int, [_CTX, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ur_beamform", C.c_int, [_CTX, P(GridDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ur_beamform_static", C.c_int, [_CTX, P(GridDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    ("ur_last_kernel_ms", C.c_int, [_CTX, P(C.c_double), P(C.c_double)]),
    ("ur_last_trace_kernels_ms", C.c_int, [_CTX, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_int64)]),
    ("ur_trace_rays", C.c_int, [_CTX, C.c_uint64, P(Ray), C.c_int64, P(Event), C.c_int64, P(C.c_int64),
                                C.c_void_p, C.c_void_p]),
    ("ur_philox", C.c_int, [_CTX, P(C.c_uint32), C.c_int64, C.c_uint32, C.c_uint32, P(C.c_uint32)]),
    ("ur_mlp_init", C.c_int, [_CTX, P(C.c_float), P(C.c_float)]),
    ("ur_mlp_get_params", C.c_int, [_CTX, P(C.c_float)]),
    ("ur_mlp_get_state", C.c_int, [_CTX, P(C.c_float), P(C.c_int64)]),
    ("ur_mlp_set_state", C.c_int, [_CTX, P(C.c_float), C.c_int64]),
    ("ur_mlp_forward", C.c_int, [_CTX, C.c_void_p, C.c_void_p]),
    ("ur_mlp_loss_grad", C.c_int, [_CTX, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ur_mlp_train_step", C.c_int, [_CTX, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p]),
    ("ur_mlp_proposal_tables", C.c_int, [_CTX, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ur_set_record", C.c_int, [_CTX, C.c_void_p, C.c_int64, C.c_void_p]),
    ("ur_record_histogram", C.c_int, [_CTX, C.c_void_p, C.c_int64, C.c_int64, C.c_uint64, C.c_uint32, C.c_void_p,
                                      C.c_void_p]),
    ("ur_set_cost_histogram", C.c_int, [_CTX, C.c_void_p]),
    ("ur_record_reweight", C.c_int, [_CTX, C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_void_p]),
    ("ur_scene_update", C.c_int, [_CTX, P(C.c_double), P(C.c_double), P(C.c_double)]),
    ("ur_pulse_adjoint", C.c_int, [_CTX, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ur_beamform_adjoint", C.c_int, [_CTX, P(GridDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    ("ur_trace_adjoint", C.c_int, [_CTX, C.c_uint64, C.c_int64, C.c_int64, C.c_void_p, P(GradDesc), C.c_void_p]),
    ("ur_set_binning", C.c_int, [_CTX, C.c_int32, C.c_int64]),
    ("ur_trace_grad_edges", C.c_int, [_CTX, C.c_uint64, C.c_int64, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
]

_lib = None


def load(path: str = None):
    """Loads libultraray.so and declares every entry point.  Raises if missing."""
    global _lib
    if path is None:
        # ULTRARAY_LIB names another build of the library (e.g. an installed copy)
        path = os.environ.get("ULTRARAY_LIB", LIB_PATH)
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes this library bind to that runtime instead of a second copy
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built: run __graft_entry__.build() (the HIP library is required; "
                              "there is no CPU fallback)")
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class URError(RuntimeError):
    pass


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


class Context:
    """One library context on one GPU; methods mirror the C entry points."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.ur_context_create(int(device), C.byref(h))
        if rc != 0:
            msg = self.lib.ur_last_error(None).decode()
            raise URError(f"ur_context_create failed: {STATUS.get(rc, rc)}: {msg}")
        self.h = h
        self.device = device
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.ur_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, what):
        if rc != 0:
            msg = self.lib.ur_last_error(self.h).decode()
            raise URError(f"{what}: {STATUS.get(rc, rc)}: {msg}")

    # ---------------------------------------------------------------- scene
    def ur_scene_upload(self, scene):
        keep = []

        def f64(x, n):
            a = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, n))
            keep.append(a)
            return a

        def i32(x):
            a = np.ascontiguousarray(np.asarray(x, np.int32).reshape(-1, 2))
            keep.append(a)
            return a

        mat, tri, sph, pln, scat = (f64(scene.materials, 3), f64(scene.tri, 9), f64(scene.sph, 4),
                                    f64(scene.pln, 4), f64(scene.scat, 4))
        box = f64(scene.box, 6)
        dp = lambda a: a.ctypes.data_as(P(C.c_double))
        ip = lambda a: a.ctypes.data_as(P(C.c_int32))
        d = SceneDesc(n_mat=len(mat), n_tri=len(tri), n_sph=len(sph), n_pln=len(pln), n_scat=len(scat),
                      top_medium=int(scene.top_medium), mat=dp(mat), box=dp(box), tri=dp(tri),
                      tri_mat=ip(i32(scene.tri_mat)), sph=dp(sph), sph_mat=ip(i32(scene.sph_mat)), pln=dp(pln),
                      pln_mat=ip(i32(scene.pln_mat)), scat=dp(scat))
        rough = getattr(scene, "rough", None)
        if rough is not None:
            rough = np.ascontiguousarray(np.asarray(rough, np.float64).reshape(-1))
            d.rough = dp(rough)
        self.check(self.lib.ur_scene_upload(self.h, C.byref(d)), "ur_scene_upload")
        self.scene_sizes = {"mat": 3 * len(mat), "scat_amp": len(scat), "sph": 4 * len(sph)}

    def ur_transmit_setup(self, acq):
        ang = np.ascontiguousarray(np.asarray(acq.angles, np.float64))
        p = ProbeDesc(n_elements=acq.n_elements, pitch=acq.pitch, elevation=acq.elevation, f_c=acq.f_c,
                      radius=float(getattr(acq, "radius", 0.0)))
        a = AcqDesc(n_tx=len(ang), n_samples=acq.n_samples, rays_per_element=acq.rays_per_element,
                    max_bounces=acq.max_bounces, binning=acq.binning, f_s=acq.f_s, c0=acq.c0,
                    n_cycles=acq.n_cycles, r_s=acq.r_s, max_path=acq.max_path, alpha_m=acq.alpha_m,
                    alpha_c=acq.alpha_c, angles=ang.ctypes.data_as(P(C.c_double)),
                    element_choice=int(getattr(acq, "element_choice", 0)), scheme=int(getattr(acq, "scheme", 0)),
                    rough_direct_only=int(getattr(acq, "rough_direct_only", 0)))
        self.check(self.lib.ur_transmit_setup(self.h, C.byref(p), C.byref(a)), "ur_transmit_setup")
        self.acq = acq

    def ur_set_proposal(self, pdf=None, cdf=None):
        self._keep = [pdf, cdf]
        self.check(self.lib.ur_set_proposal(self.h, _ptr(pdf), _ptr(cdf)), "ur_set_proposal")

    # ---------------------------------------------------------------- hot path
    def ur_trace(self, seed, ch_raw, ch_rf=None, stats=False, ray_stride=1, ray_offset=0, stream=None):
        st = TraceStats() if stats else None
        rc = self.lib.ur_trace(self.h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(ray_stride), int(ray_offset),
                               _ptr(ch_raw), _ptr(ch_rf), C.byref(st) if st is not None else None,
                               _stream_ptr(stream))
        self.check(rc, "ur_trace")
        return st.as_dict() if st is not None else None

    def ur_set_limits(self, rays_per_launch, nee_queue_capacity):
        self.check(self.lib.ur_set_limits(self.h, int(rays_per_launch), int(nee_queue_capacity)), "ur_set_limits")

    def ur_set_segment_queue(self, segments):
        self.check(self.lib.ur_set_segment_queue(self.h, int(segments)), "ur_set_segment_queue")

    def ur_pulse(self, ch_raw, ch_rf, stream=None):
        self.check(self.lib.ur_pulse(self.h, _ptr(ch_raw), _ptr(ch_rf), _stream_ptr(stream)), "ur_pulse")

    def ur_beamform(self, grid, ch_rf, iq=None, env=None, bmode=None, apod=UR_APOD_HANN, dynamic_range_db=90.0,
                    stream=None):
        g = _grid_desc(grid, apod, dynamic_range_db)
        rc = self.lib.ur_beamform(self.h, C.byref(g), _ptr(ch_rf), _ptr(iq), _ptr(env), _ptr(bmode),
                                  _stream_ptr(stream))
        self.check(rc, "ur_beamform")

    def ur_beamform_static(self, grid, ch_rf, iq=None, env=None, bmode=None, apod=UR_APOD_HANN,
                           dynamic_range_db=90.0, stream=None):
        g = _grid_desc(grid, apod, dynamic_range_db)
        rc = self.lib.ur_beamform_static(self.h, C.byref(g), _ptr(ch_rf), _ptr(iq), _ptr(env), _ptr(bmode),
                                         _stream_ptr(stream))
        self.check(rc, "ur_beamform_static")

    def ur_set_cost_histogram(self, cost):
        self.check(self.lib.ur_set_cost_histogram(self.h, _ptr(cost)), "ur_set_cost_histogram")

    def ur_record_reweight(self, rec, n_rec, cost, rays_per_row, stream=None):
        self.check(self.lib.ur_record_reweight(self.h, _ptr(rec), int(n_rec), _ptr(cost), float(rays_per_row),
                                               _stream_ptr(stream)), "ur_record_reweight")

    def ur_scene_update(self, mat=None, scat_amp=None, sph=None):
        keep = []

        sizes = getattr(self, "scene_sizes", None)
        if sizes is None:
            raise URError("ur_scene_update: upload a scene first")

        def arr(a, name):
            if a is None:
                return None
            a = np.ascontiguousarray(a, np.float64).ravel()
            if a.size != sizes[name]:
                raise URError(f"ur_scene_update: {name} has {a.size} values, the scene needs {sizes[name]}")
            keep.append(a)
            return a.ctypes.data_as(P(C.c_double))
        self.check(self.lib.ur_scene_update(self.h, arr(mat, "mat"), arr(scat_amp, "scat_amp"), arr(sph, "sph")), "ur_scene_update")

    def ur_pulse_adjoint(self, g_rf, g_raw, stream=None):
        self.check(self.lib.ur_pulse_adjoint(self.h, _ptr(g_rf), _ptr(g_raw), _stream_ptr(stream)), "ur_pulse_adjoint")

    def ur_beamform_adjoint(self, grid, g_rf, iq=None, g_env=None, g_iq=None, apod=UR_APOD_HANN, stream=None):
        g = _grid_desc(grid, apod, 90.0)
        rc = self.lib.ur_beamform_adjoint(self.h, C.byref(g), _ptr(iq), _ptr(g_env), _ptr(g_iq), _ptr(g_rf),
                                          _stream_ptr(stream))
        self.check(rc, "ur_beamform_adjoint")

    def ur_trace_adjoint(self, seed, g_raw, amp=None, alpha=None, Z=None, sph_center=None, value=None,
                         frozen_choice=False, ray_stride=1, ray_offset=0, record_paths=0, stream=None):
        d = GradDesc(amp=_ptr(amp), alpha=_ptr(alpha), Z=_ptr(Z), sph_center=_ptr(sph_center), value=_ptr(value),
                     frozen_choice=1 if frozen_choice else 0, record_paths=int(record_paths))
        rc = self.lib.ur_trace_adjoint(self.h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(ray_stride),
                                       int(ray_offset), _ptr(g_raw), C.byref(d), _stream_ptr(stream))
        self.check(rc, "ur_trace_adjoint")

    def ur_set_binning(self, deterministic, capacity=1 << 24):
        self.check(self.lib.ur_set_binning(self.h, 1 if deterministic else 0, int(capacity)), "ur_set_binning")

    def ur_trace_grad_edges(self, seed, g_raw, Z=None, sph_center=None, n_scan=16, ray_stride=1, ray_offset=0,
                            stream=None):
        rc = self.lib.ur_trace_grad_edges(self.h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(ray_stride),
                                          int(ray_offset), _ptr(g_raw), int(n_scan), _ptr(Z), _ptr(sph_center),
                                          _stream_ptr(stream))
        self.check(rc, "ur_trace_grad_edges")

    def ur_scan_convert(self, sector, img, cart, out, fill=0.0, stream=None):
        gs, gc = _grid_desc(sector, UR_APOD_NONE, 90.0), _grid_desc(cart, UR_APOD_NONE, 90.0)
        self.check(self.lib.ur_scan_convert(self.h, C.byref(gs), _ptr(img), C.byref(gc), float(fill), _ptr(out),
                                            _stream_ptr(stream)), "ur_scan_convert")

    def ur_synthesize(self, ch_sa, angles, out, stream=None):
        ang = np.ascontiguousarray(np.asarray(angles, np.float64))
        self.check(self.lib.ur_synthesize(self.h, _ptr(ch_sa), ang.ctypes.data_as(P(C.c_double)), len(ang), _ptr(out),
                                          _stream_ptr(stream)), "ur_synthesize")

    def ur_last_kernel_ms(self):
        a, b = C.c_double(), C.c_double()
        self.check(self.lib.ur_last_kernel_ms(self.h, C.byref(a), C.byref(b)), "ur_last_kernel_ms")
        return a.value, b.value

    def ur_last_trace_kernels_ms(self):
        """(extend_ms, scatter_ms, sampling_ms, launch_ranges) of the last trace."""
        a, b, c, n = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        self.check(self.lib.ur_last_trace_kernels_ms(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(n)),
                   "ur_last_trace_kernels_ms")
        return a.value, b.value, c.value, n.value

    def ur_trace_rays(self, seed, rays, cap=4096, ch_raw=None, stream=None):
        arr = (Ray * max(1, len(rays)))()
        for i, r in enumerate(rays):
            arr[i].o[:] = [float(v) for v in r["o"]]
            arr[i].d[:] = [float(v) for v in r["d"]]
            arr[i].w = float(r.get("w", 1.0))
            arr[i].t = float(r.get("t", 0.0))
            arr[i].tx = int(r.get("tx", 0))
            arr[i].elem = int(r.get("elem", 0))
            arr[i].ray = int(r.get("ray", 0))
            arr[i].medium = int(r.get("medium", 0))
        ev = (Event * max(1, cap))()
        n = C.c_int64(0)
        rc = self.lib.ur_trace_rays(self.h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), arr, len(rays), ev, cap,
                                    C.byref(n), _ptr(ch_raw), _stream_ptr(stream))
        self.check(rc, "ur_trace_rays")
        return [dict(kind=EVENT_KINDS[ev[i].kind], tx=ev[i].tx, elem=ev[i].elem, seg=ev[i].seg, id=ev[i].id,
                     t=ev[i].t, value=ev[i].value, pos=(ev[i].x, ev[i].y, ev[i].z))
                for i in range(min(n.value, cap))], n.value

    def ur_philox(self, ctr, key0, key1):
        c = np.ascontiguousarray(np.asarray(ctr, np.uint32).reshape(-1, 4))
        out = np.zeros_like(c)
        rc = self.lib.ur_philox(self.h, c.ctypes.data_as(P(C.c_uint32)), len(c), int(key0) & 0xFFFFFFFF,
                                int(key1) & 0xFFFFFFFF, out.ctypes.data_as(P(C.c_uint32)))
        self.check(rc, "ur_philox")
        return out

    # ---------------------------------------------------------- proposal network
    def ur_mlp_init(self, params, rff):
        p = np.ascontiguousarray(np.asarray(params, np.float32).ravel())
        b = np.ascontiguousarray(np.asarray(rff, np.float32).ravel())
        if p.size != 77120 or b.size != 32:
            raise ValueError("need 77120 parameters and a 16x2 Fourier matrix")
        self.check(self.lib.ur_mlp_init(self.h, p.ctypes.data_as(P(C.c_float)), b.ctypes.data_as(P(C.c_float))),
                   "ur_mlp_init")

    def ur_mlp_get_params(self):
        out = np.zeros(77120, np.float32)
        self.check(self.lib.ur_mlp_get_params(self.h, out.ctypes.data_as(P(C.c_float))), "ur_mlp_get_params")
        return out

    def ur_mlp_get_state(self):
        """(state [3][77120] float32: parameters, Adam m, Adam v; step)."""
        out = np.zeros(3 * 77120, np.float32)
        step = C.c_int64(0)
        self.check(self.lib.ur_mlp_get_state(self.h, out.ctypes.data_as(P(C.c_float)), C.byref(step)),
                   "ur_mlp_get_state")
        return out.reshape(3, 77120), int(step.value)

    def ur_mlp_set_state(self, state, step):
        a = np.ascontiguousarray(state, np.float32).reshape(-1)
        if a.size != 3 * 77120:
            raise ValueError("state must hold 3 x 77120 floats")
        self.check(self.lib.ur_mlp_set_state(self.h, a.ctypes.data_as(P(C.c_float)), int(step)), "ur_mlp_set_state")

    def ur_mlp_forward(self, q, stream=None):
        self.check(self.lib.ur_mlp_forward(self.h, _ptr(q), _stream_ptr(stream)), "ur_mlp_forward")

    def ur_mlp_loss_grad(self, hist, grad, loss=None, stream=None):
        self.check(self.lib.ur_mlp_loss_grad(self.h, _ptr(hist), _ptr(grad), _ptr(loss), _stream_ptr(stream)),
                   "ur_mlp_loss_grad")

    def ur_mlp_train_step(self, hist, lr, loss=None, stream=None):
        self.check(self.lib.ur_mlp_train_step(self.h, _ptr(hist), float(lr), _ptr(loss), _stream_ptr(stream)),
                   "ur_mlp_train_step")

    def ur_mlp_proposal_tables(self, eps, pdf, cdf, stream=None):
        self.check(self.lib.ur_mlp_proposal_tables(self.h, float(eps), _ptr(pdf), _ptr(cdf), _stream_ptr(stream)),
                   "ur_mlp_proposal_tables")

    def ur_set_record(self, rec=None, count=None):
        cap = rec.numel() // 2 if rec is not None else 0
        self.check(self.lib.ur_set_record(self.h, _ptr(rec), int(cap), _ptr(count)), "ur_set_record")

    def ur_record_histogram(self, rec, n_rec, batch, seed, step, hist, stream=None):
        self.check(self.lib.ur_record_histogram(self.h, _ptr(rec), int(n_rec), int(batch),
                                                C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(step) & 0xFFFFFFFF,
                                                _ptr(hist), _stream_ptr(stream)), "ur_record_histogram")

