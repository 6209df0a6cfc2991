"""The C ABI on the host (no GPU): the library loads, exports exactly the
entry points include/ultraray.h declares, the Python binding declares each
of them, and the ctypes struct layouts match the C header's."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ultraray.h")


def declared():
    src = open(HEADER).read()
    return re.findall(r"UR_API\s+[\w\s\*]+?\b(ur_\w+)\s*\(", src)


def test_header_declares_entry_points():
    names = declared()
    for n in ["ur_context_create", "ur_scene_upload", "ur_transmit_setup", "ur_trace", "ur_pulse", "ur_beamform",
              "ur_set_proposal", "ur_trace_rays", "ur_philox", "ur_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2501_05828_amd import binding
    lib = binding.load()
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ur_\w+)", out))
    assert exported == set(declared())
    assert {s[0] for s in binding.SIGNATURES} == set(declared())
    assert lib.ur_version().startswith(b"ultraray")


def test_struct_layouts_match_header(tmp_path):
    from paper_2501_05828_amd import binding as B
    import ctypes
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ultraray.h"\nint main(void){\n'
                    'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ur_scene_desc),'
                    ' sizeof(ur_probe_desc), sizeof(ur_acq_desc), sizeof(ur_grid_desc), sizeof(ur_trace_stats),'
                    ' sizeof(ur_event), sizeof(ur_ray), offsetof(ur_trace_stats, kernel_ms),'
                    ' offsetof(ur_acq_desc, angles), sizeof(ur_grad_desc), offsetof(ur_grad_desc, frozen_choice),'
                    ' offsetof(ur_grad_desc, record_paths));\n'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    want = [ctypes.sizeof(B.SceneDesc), ctypes.sizeof(B.ProbeDesc), ctypes.sizeof(B.AcqDesc),
            ctypes.sizeof(B.GridDesc), ctypes.sizeof(B.TraceStats), ctypes.sizeof(B.Event), ctypes.sizeof(B.Ray),
            B.TraceStats.kernel_ms.offset, B.AcqDesc.angles.offset, ctypes.sizeof(B.GradDesc),
            B.GradDesc.frozen_choice.offset, B.GradDesc.record_paths.offset]
    assert got == want


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2501_05828_amd import binding
    # the failing HIP call is named although no context exists
    with pytest.raises(binding.URError, match="hipGetDeviceCount"):
        binding.Context(0)
