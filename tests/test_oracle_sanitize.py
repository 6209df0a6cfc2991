"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a child process with libasan preloaded runs the oracle's entry
points on small cases -- plane-wave and synthetic-aperture traces with both
binnings, a convex array, a rough floor with transducer sampling, explicit
rays with their event log, the forward-mode gradient (frozen and attached
choice), pulse and DAS -- and any report (every one is fatal) fails it."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = r"""
import dataclasses, math, sys
import numpy as np
sys.path.insert(0, ROOT)
from paper_2501_05828_amd import scenes
from oracle import oracle as o

w = scenes.tiny(rays_per_element=16)
ch, st = o.trace(w)
assert st["rays"] == 16 * 64 and np.isfinite(ch).all()
wl = dataclasses.replace(w, acq=dataclasses.replace(w.acq, binning=scenes.LINEAR, alpha_c=math.radians(30)))
o.trace(wl, ray_stride=3)
o.trace(scenes.synthetic_aperture(scenes.tiny(rays_per_element=4)), ray_stride=8)
o.trace(scenes.tiny_convex(rays_per_element=8))
rough = dataclasses.replace(w.scene, rough=np.array([0.0, 0.5, 0.0]))        # the reflector rough
o.trace(dataclasses.replace(w, scene=rough, acq=dataclasses.replace(w.acq, rough_direct_only=0)))
rays = [dict(o=(0.0, 0.0, 0.0), d=(0.0, 0.3, math.sqrt(1 - 0.09)), w=1.0, t=0.0, ray=r, elem=r % 64) for r in range(20)]
ev, st, _ = o.trace_rays(w, rays, cap=500)
assert len(ev) > 0
g = np.random.default_rng(1).normal(size=(w.acq.n_tx, w.acq.n_elements, w.acq.n_samples))
for attach in (False, True):
    r = o.trace_grad(wl, g, attach_choice=attach, ray_stride=4)
    assert np.isfinite(r["J"])
raw = np.random.default_rng(2).normal(size=(w.acq.n_tx, w.acq.n_elements, w.acq.n_samples))
rf = o.pulse(w.acq, raw)
img = o.das(w.acq, dataclasses.replace(w.grid, nx=16, nz=16), rf)
assert np.isfinite(img).all()
maps = open("/proc/self/maps").read()
assert "libasan" in maps and "liboracle_san" in maps, "the sanitizer runtime or the sanitized oracle is not loaded"
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    from oracle import oracle
    try:
        asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("gcc is not available")
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not installed")
    lib = oracle.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib, OMP_NUM_THREADS="1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sys.executable, "-c", "ROOT = %r\n" % ROOT + SCRIPT], env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "sanitized oracle ok" in out
