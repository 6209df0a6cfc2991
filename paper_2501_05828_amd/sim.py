"""Device-resident simulation of one workload through the C ABI.

Allocates the channel-data and image buffers as torch tensors on the GPU
and calls the library's entry points on torch's current stream.
"""
from __future__ import annotations

import torch

from . import binding


class Simulator:
    def __init__(self, workload, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP GPU is required")
        self.w = workload
        self.dev = torch.device("cuda", device)
        self.ctx = binding.Context(device)
        self.ctx.ur_scene_upload(workload.scene)
        self.ctx.ur_transmit_setup(workload.acq)
        a = workload.acq
        shape = (a.n_tx, a.n_elements, a.n_samples)
        self.ch_raw = torch.empty(shape, dtype=torch.float32, device=self.dev)
        self.ch_rf = torch.empty(shape + (2,), dtype=torch.float32, device=self.dev)
        g = workload.grid
        self.iq = torch.empty((g.nx, g.nz, 2), dtype=torch.float32, device=self.dev)
        self.env = torch.empty((g.nx, g.nz), dtype=torch.float32, device=self.dev)
        self.bmode = torch.empty((g.nx, g.nz), dtype=torch.float32, device=self.dev)
        # a sector image is scan converted to its Cartesian display grid
        self.cart_grid = workload.extra.get("cart_grid") if getattr(g, "sector", False) else None
        self.cart = None
        if self.cart_grid is not None:
            self.cart = torch.empty((self.cart_grid.nx, self.cart_grid.nz), dtype=torch.float32, device=self.dev)

    def set_acquisition(self, acq):
        self.ctx.ur_transmit_setup(acq)
        self.w.acq = acq

    def trace(self, seed=None, stats=False, ray_stride=1, ray_offset=0, pulse=True):
        seed = self.w.seed if seed is None else seed
        return self.ctx.ur_trace(seed, self.ch_raw, self.ch_rf if pulse else None, stats=stats,
                                 ray_stride=ray_stride, ray_offset=ray_offset)

    def beamform(self, bmode=True, dynamic_range_db=90.0):
        apod = binding.UR_APOD_HANN if self.w.apod == "hann" else binding.UR_APOD_NONE
        self.ctx.ur_beamform(self.w.grid, self.ch_rf, iq=self.iq, env=self.env,
                             bmode=self.bmode if bmode else None, apod=apod, dynamic_range_db=dynamic_range_db)

    def scan_convert(self, dynamic_range_db=90.0):
        self.ctx.ur_scan_convert(self.w.grid, self.bmode, self.cart_grid, self.cart, fill=-dynamic_range_db)

    def step(self, seed=None):
        """One pass of the hot path: trace + bin, pulse, DAS, envelope, log
        (and, on a sector grid, scan conversion of the B-mode image)."""
        self.trace(seed)
        self.beamform()
        if self.cart is not None:
            self.scan_convert()
        return self.env

    def kernel_ms(self):
        return self.ctx.ur_last_kernel_ms()
