"""The device code is built without packed FP32 instructions (CPU only).

hipcc for gfx950 turns ordinary float2 / paired float arithmetic into
v_pk_{add,mul,fma}_f32 unless the target feature packed-fp32-ops is
switched off.  The library's build line switches it off (the host pass of
hipcc warns that it does not know the feature, which is expected: the
feature belongs to the device pass).  These tests compile device code only
(no GPU needed) and read the gfx950 assembly of our own sources."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

from paper_2506_03266_amd import build

HIPCC = "/opt/rocm/bin/hipcc"
FEATURE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")


def device_asm(src_path, flags, out):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-S", "-o", out,
           "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC] + flags + [src_path]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read()


def test_build_line_switches_packed_fp32_off():
    flags = build.HIPCC_FLAGS
    i = flags.index("-target-feature")
    assert flags[i - 1] == "-Xclang" and flags[i + 1] == "-Xclang" and flags[i + 2] == "-packed-fp32-ops"


def test_feature_removes_packed_fp32_on_the_device(tmp_path):
    probe = os.path.join(tmp_path, "probe.hip")
    with open(probe, "w") as f:
        f.write("#include <hip/hip_runtime.h>\n"
                "__global__ void k(float2 *a, const float2 *b, float s) {\n"
                "  int i = threadIdx.x; float2 x = a[i], y = b[i];\n"
                "  x.x = x.x * s + y.x; x.y = x.y * s + y.y; a[i] = x; }\n")
    on = device_asm(probe, [], os.path.join(tmp_path, "on.s"))
    off = device_asm(probe, FEATURE, os.path.join(tmp_path, "off.s"))
    assert PACKED.search(on), "the probe no longer produces packed FP32; pick a probe that does"
    assert not PACKED.search(off)


@pytest.mark.slow
@pytest.mark.parametrize("src", build.SOURCES)
def test_library_has_no_packed_fp32(tmp_path, src):
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    flags = [f for f in flags if not f.startswith("--offload-arch")]
    asm = device_asm(os.path.join(build.CSRC, src), flags, os.path.join(tmp_path, src + ".s"))
    m = PACKED.search(asm)
    assert m is None, f"{src}: {m.group(0)} in the gfx950 code"
