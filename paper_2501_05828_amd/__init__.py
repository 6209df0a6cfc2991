"""MI355X-native full-path ultrasound ray tracer (UltraRay, arXiv 2501.05828).

The simulation runs in the HIP library libultraray.so (C ABI in
include/ultraray.h); `binding` marshals arguments, `sim` wraps a context with
torch-allocated device buffers, `scenes` builds seeded synthetic workloads.
"""
from . import scenes  # noqa: F401


def __getattr__(name):
    if name in ("binding", "sim"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    if name in ("Simulator",):
        from .sim import Simulator
        return Simulator
    raise AttributeError(name)
